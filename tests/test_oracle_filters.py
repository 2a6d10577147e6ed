"""Pins of the oracle's filter steps against what the paper and mathematics fix.

* Linear-Gaussian workload: the Kalman filter is the exact posterior; the
  look-ahead DPF and the DPF must approach it as N and M grow, and their
  evidence estimates must approach the Kalman log-likelihood.
* The inner cloud of a single outer particle must approach the exact
  conditional filter of z given the x path -- on the coupled model this
  exercises the x-conditioning of eq:qnobar.
* The look-ahead weight (eq:weightsMC) has a closed-form expectation on the
  linear-Gaussian model; the SIR-selected x (eq:approx3) has the closed-form
  optimal proposal (eq:optdistbayes) as its law.
* Brute force over every resampling outcome of a tiny filter gives the exact
  expectation of the new x, which must equal the Rao-Blackwellised estimate.
* With one inner particle the DPF is the textbook bootstrap particle filter
  on the joint (x, z) space.
"""
import math

import numpy as np
import pytest
from scipy import stats

import dpf_synth as S
from oracle import dpf, kalman, ladpf
from oracle import philox as P
from oracle.models import make_model


def _model(spec):
    return make_model(spec.kind, spec.dx, spec.dz, spec.dy, spec.blob)


def _kf_errors(run_out, mu):
    ex = np.mean(np.abs(run_out["xhat"][:, 0] - mu[:, 0]))
    ez = np.mean(np.abs(run_out["zhat"] - mu[:, 1:]))
    return ex, ez


@pytest.mark.slow
@pytest.mark.parametrize("coupled", [False, True])
def test_ladpf_converges_to_kalman(coupled):
    spec = S.lingauss_c1(coupled)
    m = _model(spec)
    T = 30
    _, _, ys = S.simulate(spec, T, 11)
    mu, Pk, ll = kalman.kalman_filter(m, ys)
    errs, lls = [], []
    for N, M in [(10, 5), (60, 30), (300, 100)]:
        e = []
        for rep in range(2):
            out = ladpf.run(m, N, M, ys, seed=1000 + rep, fid=rep)
            e.append(_kf_errors(out, mu))
            lls.append((N * M, out["dlogz"].sum()))
        errs.append(np.mean(e, axis=0))
    errs = np.array(errs)
    assert np.all(np.diff(errs[:, 0]) < 0) and np.all(np.diff(errs[:, 1]) < 0)
    # at the largest size the error is a small fraction of the posterior std
    assert errs[-1, 0] < 0.1 * np.sqrt(Pk[:, 0, 0]).mean()
    # evidence: log Z within a few tenths of the Kalman log-likelihood
    assert all(abs(v - ll) < 1.0 for nm, v in lls if nm >= 30000)


@pytest.mark.slow
def test_plain_dpf_converges_to_kalman():
    spec = S.lingauss_c1(True)
    m = _model(spec)
    _, _, ys = S.simulate(spec, 30, 12)
    mu, Pk, ll = kalman.kalman_filter(m, ys)
    errs = []
    for N, M in [(10, 5), (300, 100)]:
        out = dpf.run(m, N, M, ys, seed=5, fid=0)
        errs.append(_kf_errors(out, mu))
    assert errs[1][0] < errs[0][0] and errs[1][1] < errs[0][1]
    assert errs[1][0] < 0.15 * np.sqrt(Pk[:, 0, 0]).mean()
    assert abs(out["dlogz"].sum() - ll) < 1.5


def test_inner_cloud_matches_conditional_kalman():
    """N = 1: no outer resampling; the inner cloud must track p(z_t | x_{0:t}, y_{1:t})."""
    spec = S.lingauss_c1(True)
    m = _model(spec)
    _, _, ys = S.simulate(spec, 12, 3)
    M = 40000
    state = ladpf.init_state(m, 1, M, 77, 0)
    mu_c, P_c = np.zeros(2), np.eye(2)
    for y in ys:
        x_prev = state["x"][0].copy()
        state, info = ladpf.step(m, state, y, 77, 0)
        mu_c, P_c = kalman.conditional_kf_step(m, mu_c, P_c, x_prev, state["x"][0], y)
        q = np.exp(state["lam"][0])
        zbar = q @ state["z"][0]
        cov = (state["z"][0] - zbar).T @ ((state["z"][0] - zbar) * q[:, None])
        ess = 1.0 / np.sum(q * q)
        se = np.sqrt(np.diag(P_c) / ess)
        assert np.all(np.abs(zbar - mu_c) < 6 * se + 1e-3)
        assert np.allclose(np.diag(cov), np.diag(P_c), rtol=0.1)


def test_inner_kalman_pin_detects_missing_x_conditioning():
    """Dropping the eq:qnobar factor must break the conditional-filter pin."""
    spec = S.lingauss_c1(True)
    m = _model(spec)
    _, _, ys = S.simulate(spec, 6, 3)
    M = 40000
    state = ladpf.init_state(m, 1, M, 77, 0)
    real = m.logpx
    m.logpx = lambda xn, x, z, t=0: np.zeros(np.broadcast(xn[..., 0], z[..., 0]).shape)
    mu_c, P_c = np.zeros(2), np.eye(2)
    worst = 0.0
    for y in ys:
        x_prev = state["x"][0].copy()
        state, _ = ladpf.step(m, state, y, 77, 0)
        mu_c, P_c = kalman.conditional_kf_step(m, mu_c, P_c, x_prev, state["x"][0], y)
        q = np.exp(state["lam"][0])
        zbar = q @ state["z"][0]
        se = np.sqrt(np.diag(P_c) / (1.0 / np.sum(q * q)))
        worst = max(worst, float(np.max(np.abs(zbar - mu_c) / (6 * se + 1e-3))))
    m.logpx = real
    assert worst > 1.0


def _random_state(m, N, M, g):
    lam = g.normal(size=(N, M))
    lam -= np.log(np.exp(lam).sum(axis=1, keepdims=True))
    return {"x": g.normal(size=(N, m.dx)), "z": g.normal(size=(N, M, m.dz)), "lam": lam, "t": 4}


def test_lookahead_weight_expectation_closed_form():
    """E[w_i] = sum_j qbar_j N(y; 1.575 x + 0.8 z1_j + 0.45 z2_j, 0.63125)."""
    spec = S.lingauss_c1(False)
    m = _model(spec)
    g = np.random.default_rng(5)
    st = _random_state(m, 3, 4, g)
    y = np.array([0.4])
    R = 4000
    W = np.empty((R, 3))
    for r in range(R):
        _, _, _, logw = ladpf.lookahead(m, st, y, 99, r)
        W[r] = np.exp(logw)
    qbar = np.exp(st["lam"])
    mj = 1.575 * st["x"][:, :1] + 0.8 * st["z"][:, :, 0] + 0.45 * st["z"][:, :, 1]
    expect = np.sum(qbar * stats.norm.pdf(y[0], mj, math.sqrt(0.63125)), axis=1)
    se = W.std(axis=0) / math.sqrt(R)
    assert np.all(np.abs(W.mean(axis=0) - expect) < 5 * se)


def test_candidate_law_is_optimal_proposal():
    """SIR over look-ahead candidates draws from the optimal proposal mixture."""
    spec = S.lingauss_c1(False)
    m = _model(spec)
    g = np.random.default_rng(6)
    N, M = 2000, 400
    x0 = 0.3
    zc = g.normal(size=(M, 2)) * 0.7
    state = {"x": np.full((N, 1), x0), "z": np.broadcast_to(zc, (N, M, 2)).copy(),
             "lam": np.full((N, M), -math.log(M)), "t": 2}
    y = np.array([1.1])
    new, _ = ladpf.step(m, state, y, 31, 0)
    xs = new["x"][:, 0]
    mj = 1.575 * x0 + 0.8 * zc[:, 0] + 0.45 * zc[:, 1]
    pi = stats.norm.pdf(y[0], mj, math.sqrt(0.63125))
    pi /= pi.sum()
    K = 1.75 * 0.1 / 0.63125
    mean_j = 0.9 * x0 + K * (y[0] - mj)
    sd = math.sqrt(1.0 / (1.0 / 0.1 + 1.75 ** 2 / 0.325))
    cdf = lambda v: np.sum(pi[None, :] * stats.norm.cdf((np.atleast_1d(v)[:, None] - mean_j) / sd), axis=1)
    assert stats.kstest(xs, cdf).pvalue > 1e-3
    # and it differs from the prior mixture (the look-ahead uses y_t)
    prior_cdf = lambda v: stats.norm.cdf((np.atleast_1d(v) - 0.9 * x0) / math.sqrt(0.1))
    assert stats.kstest(xs, prior_cdf).pvalue < 1e-6


def _bp_systematic(w, n_out):
    C = np.cumsum(w)
    return {c * n_out / C[-1] - k for k in range(n_out) for c in C} | {0.0, 1.0}


@pytest.mark.parametrize("N,M", [(1, 1), (1, 3), (2, 2), (2, 3), (3, 2), (3, 3)])
def test_bruteforce_expectation_equals_rao_blackwell(N, M):
    spec = S.lingauss_c1(True)
    m = _model(spec)
    g = np.random.default_rng(N * 10 + M)
    st = _random_state(m, N, M, g)
    y = np.array([0.2])
    _, info0 = ladpf.step(m, st, y, 8, 0)
    ell, xla, logw = info0["ell"], info0["xla"], info0["logw"]
    # expected value written from the definitions, not from the oracle's estimate
    W = np.exp(logw - logw.max()); W /= W.sum()
    pi = np.exp(ell - ell.max(axis=1, keepdims=True)); pi /= pi.sum(axis=1, keepdims=True)
    expect = np.einsum("n,nm,nm->", W, pi, xla[:, :, 0])
    assert np.isclose(info0["xhat_rb"][0], expect, rtol=1e-12)
    bo = np.array(sorted(b for b in _bp_systematic(np.exp(logw - logw.max()), N) if 0 <= b <= 1))
    bc = set([0.0, 1.0])
    for i in range(N):
        w = np.exp(ell[i] - ell[i].max())
        bc |= {b for b in _bp_systematic(w, 1) if 0 <= b <= 1}
    bc = np.array(sorted(bc))
    E = 0.0
    for lo, hi in zip(bo[:-1], bo[1:]):
        if hi - lo < 1e-13:
            continue
        for clo, chi in zip(bc[:-1], bc[1:]):
            if chi - clo < 1e-13:
                continue
            _, info = ladpf.step(m, st, y, 8, 0, u_outer=0.5 * (lo + hi),
                                 u_cand=np.full(N, 0.5 * (clo + chi)))
            E += (hi - lo) * (chi - clo) * info["xhat"][0]
    assert np.isclose(E, expect, rtol=1e-9, atol=1e-12)


def test_inner_weights_normalised():
    spec = S.nonlin_c2(1)
    m = _model(spec)
    _, _, ys = S.simulate(spec, 3, 1)
    out = ladpf.run(m, 20, 16, ys, seed=3, fid=2)
    assert np.allclose(np.exp(out["state"]["lam"]).sum(axis=1), 1.0, atol=1e-12)
    assert np.all(out["ess"] >= 1.0 - 1e-12) and np.all(out["ess"] <= 20 + 1e-9)


def _textbook_systematic(w, u):
    """Pointer walk over the cumulative sum (a different route to the same rule)."""
    n = len(w)
    C = np.cumsum(w)
    out = np.empty(n, dtype=np.int64)
    i = 0
    for k in range(n):
        pt = ((k + u) * C[-1]) / n
        while i < n - 1 and not C[i] > pt:
            i += 1
        out[k] = i
    return out


def test_plain_dpf_with_one_inner_particle_is_bootstrap_pf():
    spec = S.lingauss_c1(True)
    m = _model(spec)
    _, _, ys = S.simulate(spec, 15, 4)
    N, seed, fid = 64, 21, 3
    out = dpf.run(m, N, 1, ys, seed, fid)
    # Bootstrap PF on s = (x, z): propagate jointly with the transition prior,
    # weight by the likelihood, resample systematically.
    idx = np.arange(N)
    x = P.normals(seed, fid, 0, idx, 0, P.INIT_X, 1)
    z = P.normals(seed, fid, 0, idx, 0, P.INIT_Z, 2)

    def propagate(x, z, t):
        xn = m.fx(x, z, P.normals(seed, fid, t, idx, 0, P.DPF_X, 1))
        zn = m.fz(x, xn, z, P.normals(seed, fid, t, idx, 0, P.DPF_Z, 2))
        return xn, zn

    x, z = propagate(x, z, 0)
    for t, y in enumerate(ys, start=1):
        lw = m.logpy(y, x, z)
        w = np.exp(lw - lw.max())
        xhat = (w / w.sum()) @ x
        assert np.allclose(xhat, out["xhat"][t - 1], rtol=1e-12, atol=1e-14)
        A = _textbook_systematic(w, float(P.uniform53(seed, fid, t, 0, P.OUTER_U)))
        x, z = propagate(x[A], z[A], t)
    assert np.allclose(x, out["state"]["xt"], rtol=1e-12)


# ---- nested look-ahead estimator (K companions per candidate)
# Linear-Gaussian pieces written out from the model statement of the
# workload (c = [1, 0.5], A = [[0.8, 0.1], [0, 0.7]], coupling 0.2 z1 into x
# for the coupled variant): given x_{t-1} = x and one inner component z_j,
#   y_t ~ N(1.575 x + (0.8 + 1.75 g) z1 + 0.45 z2, 0.63125), g the coupling;
# given also the candidate x_t = xc,
#   y_t ~ N(1.75 xc + 0.8 z1 + 0.45 z2, 0.325)   (c.(A z + 0.5 xc 1) + xc,
#   variance c.c 0.1 + 0.2), and x_t | x, z_j ~ N(0.9 x + g z1, 0.1).
def _y_given_parent(x, z, g):
    return 1.575 * x + (0.8 + 1.75 * g) * z[..., 0] + 0.45 * z[..., 1], 0.63125


@pytest.mark.parametrize("coupled,K", [(False, 1), (False, 4), (True, 1), (True, 3)])
def test_nested_lookahead_weight_expectation_closed_form(coupled, K):
    """For any number of companions the nested weight is unbiased for the
    predictive likelihood of eq:weightsopt under the inner cloud:
    E[w_i] = sum_j qbar_j p(y_t | x_{t-1}^i, z_{t-1}^{ij}).  On the coupled
    model this needs the companions' ancestors drawn from the inner weights
    conditioned on the candidate (eq:qnobar)."""
    spec = S.lingauss_c1(coupled)
    m = _model(spec)
    g = np.random.default_rng(15 + K + 10 * coupled)
    st = _random_state(m, 3, 4, g)
    st["z"] *= 2.0                        # spread clouds: the conditioning matters
    y = np.array([0.9])
    R = 3000
    W = np.empty((R, 3))
    for r in range(R):
        _, _, logw, _, _ = ladpf.lookahead_nested(m, st, y, 99, r, K)
        W[r] = np.exp(logw)
    qbar = np.exp(st["lam"])
    mj, v = _y_given_parent(st["x"][:, :1], st["z"], 0.2 if coupled else 0.0)
    expect = np.sum(qbar * stats.norm.pdf(y[0], mj, math.sqrt(v)), axis=1)
    se = W.std(axis=0) / math.sqrt(R)
    assert np.all(np.abs(W.mean(axis=0) - expect) < 5 * se), (W.mean(axis=0), expect, se)


@pytest.mark.parametrize("coupled", [False, True])
def test_nested_candidate_score_with_many_companions(coupled):
    """With many companions ell^{(i,m)} - lam^{(i,m)} approaches the inner
    predictive likelihood at the candidate, log sum_j q_j N(y; 1.75 xc +
    0.8 z1_j + 0.45 z2_j, 0.325), q_j proportional to qbar_j p(xc | x, z_j)
    (eq:approx3's first factor with the x-conditioned inner weights)."""
    spec = S.lingauss_c1(coupled)
    m = _model(spec)
    gc = 0.2 if coupled else 0.0
    rng = np.random.default_rng(21)
    st = _random_state(m, 2, 3, rng)
    st["z"] *= 2.0
    y = np.array([0.5])
    K = 200000
    xla, ell, _, comp, _ = ladpf.lookahead_nested(m, st, y, 5, 0, K)
    for i in range(2):
        for j in range(3):
            xc = xla[i, j, 0]
            px = stats.norm.pdf(xc, 0.9 * st["x"][i, 0] + gc * st["z"][i, :, 0], math.sqrt(0.1))
            q = np.exp(st["lam"][i]) * px
            q /= q.sum()
            mu = 1.75 * xc + 0.8 * st["z"][i, :, 0] + 0.45 * st["z"][i, :, 1]
            ref = np.sum(q * stats.norm.pdf(y[0], mu, math.sqrt(0.325)))
            # Monte Carlo error of the mean of K likelihood values: with
            # s = c.w ~ N(0, 0.125), E_s[N(y; mu + s, 0.2)^2] =
            # N(y; mu, 0.1 + 0.125) / sqrt(0.8 pi) bounds each term's variance
            se = math.sqrt(np.sum(q * stats.norm.pdf(y[0], mu, math.sqrt(0.225))) / math.sqrt(0.8 * math.pi) / K)
            got = math.exp(ell[i, j] - st["lam"][i, j])
            assert abs(got - ref) <= 6 * se, (i, j, got, ref, se)
            # the companions' ancestors follow the conditioned weights
            cnt = np.bincount(comp[i, j], minlength=3)
            assert np.all(np.abs(cnt - K * q) <= 1.0 + 1e-9)


def test_nested_step_resamples_and_proposes_as_the_paired_step():
    """Steps 3-4 do not depend on how the weights were formed: a nested step
    on the plain linear-Gaussian model keeps the step's invariants and its
    x estimate tracks the Kalman filter like the paired reading's."""
    spec = S.lingauss_c1(False)
    m = _model(spec)
    _, _, ys = S.simulate(spec, 12, 8)
    mu, _, _ = kalman.kalman_filter(m, ys)
    out = ladpf.run(m, 60, 12, ys, 3, 0, n_comp=3)
    assert np.all(np.isfinite(out["xhat"]))
    assert np.mean(np.abs(out["xhat"][:, 0] - mu[:, 0])) < 0.15


@pytest.mark.parametrize("K", [0, 3])
def test_predicted_observation_expectation_closed_form(K):
    """The predicted observation weighs the look-ahead draws as draws from
    the one-step predictive: on the linear-Gaussian model its expectation
    over the draws is (1/N) sum_i sum_j qbar_ij (1.575 x_i + 0.8 z1_ij +
    0.45 z2_ij) (y = x + [1, .5] z with x_t = .9 x + v, z_t = A z + .5 x_t 1 + w),
    for the paired draws and for K companions per candidate."""
    spec = S.lingauss_c1(False)
    m = _model(spec)
    g = np.random.default_rng(33 + K)
    st = _random_state(m, 4, 5, g)
    y = np.array([0.3])
    R = 1500
    Y = np.empty(R)
    for r in range(R):
        _, info = ladpf.step(m, st, y, 17, r, n_comp=K)
        Y[r] = info["yhat"][0]
    mj, _ = _y_given_parent(st["x"][:, :1], st["z"], 0.0)
    expect = np.sum(np.exp(st["lam"]) * mj) / 4
    se = Y.std() / math.sqrt(R)
    assert abs(Y.mean() - expect) < 5 * se, (Y.mean(), expect, se)


def test_predicted_observation_approaches_the_kalman_prediction():
    """With many particles yhat_{t|t-1} approaches the Kalman filter's
    one-step prediction H F mu_{t-1}."""
    spec = S.lingauss_c1(False)
    m = _model(spec)
    _, _, ys = S.simulate(spec, 6, 4)
    F, Q, H, R_ = kalman.joint_matrices(m)
    mu, _, _ = kalman.kalman_filter(m, ys)
    st = ladpf.init_state(m, 3000, 40, 8, 0)
    errs = []
    for t in range(6):
        st, info = ladpf.step(m, st, ys[t], 8, 0)
        pred = (H @ F @ mu[t - 1])[0] if t > 0 else 0.0
        errs.append(abs(info["yhat"][0] - pred))
    assert max(errs) < 0.05, errs
