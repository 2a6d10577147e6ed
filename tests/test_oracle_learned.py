"""Pins of the learned-proposal oracle (CPU only).

Gradients against central finite differences and against torch autograd in
FP64 (a library cross-check); GELU, the mixture density and Adam against
library implementations; BF16 rounding against exact hand cases and torch;
sampling against the mixture CDF; the learned step reduces to the bootstrap
weight when the proposal is the transition density, and falls back to the
look-ahead step bit for bit when its ESS collapses.
"""
import math

import numpy as np
import pytest
from scipy import stats

import dpf_synth as S
from oracle import ladpf
from oracle import learned as Lr
from oracle.models import make_model

torch = pytest.importorskip("torch")


def test_bf16_rounding_cases():
    one = 1.0
    assert Lr.bf16(one) == 1.0
    assert Lr.bf16(1.0 + 2 ** -8) == 1.0                 # tie -> even (1.0)
    assert Lr.bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6   # tie -> even (odd neighbour rejected)
    assert Lr.bf16(1.0 + 2 ** -8 + 2 ** -12) == 1.0 + 2 ** -7
    g = np.random.default_rng(0)
    x = g.normal(size=10000) * 10 ** g.uniform(-5, 5, size=10000)
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(Lr.bf16(x), ref)


def test_gelu_matches_torch():
    a = np.linspace(-8, 8, 1001)
    ref = torch.nn.functional.gelu(torch.tensor(a), approximate="tanh").numpy()
    assert np.allclose(Lr.gelu(a), ref, rtol=1e-14, atol=1e-15)
    ta = torch.tensor(a, requires_grad=True)
    torch.nn.functional.gelu(ta, approximate="tanh").sum().backward()
    assert np.allclose(Lr.gelu_grad(a), ta.grad.numpy(), rtol=1e-12, atol=1e-14)


def _rand_out(g, B):
    out = g.normal(size=(B, Lr.D_OUT))
    out[:, Lr.K_MIX + 2 * Lr.K_MIX:] *= 0.5
    return out


def test_mdn_logpdf_matches_scipy():
    g = np.random.default_rng(1)
    out = _rand_out(g, 7)
    x = g.normal(size=(7, 2))
    got = Lr.mdn_logpdf(out, x)
    logits, mu, s = Lr.mdn_split(out)
    for r in range(7):
        pi = np.exp(logits[r] - logits[r].max())
        pi /= pi.sum()
        dens = sum(pi[c] * stats.multivariate_normal.pdf(x[r], mu[r, c], np.diag(np.exp(2 * s[r, c])))
                   for c in range(Lr.K_MIX))
        assert np.isclose(got[r], np.log(dens), rtol=1e-12)


def test_mdn_nll_gradient_finite_differences_and_autograd():
    g = np.random.default_rng(2)
    B = 5
    out = _rand_out(g, B)
    x = g.normal(size=(B, 2))
    L, grad = Lr.mdn_nll_grad(out, x)
    assert np.isclose(L, -np.mean(Lr.mdn_logpdf(out, x)), rtol=1e-13)
    h = 1e-6
    for (r, c) in [(0, 0), (1, 3), (2, 5), (3, 12), (4, 19), (0, 15)]:
        op, om = out.copy(), out.copy()
        op[r, c] += h
        om[r, c] -= h
        fd = (Lr.mdn_nll_grad(op, x)[0] - Lr.mdn_nll_grad(om, x)[0]) / (2 * h)
        assert abs(fd - grad[r, c]) < 1e-6 * max(1.0, abs(fd))
    to = torch.tensor(out, requires_grad=True)
    logits, mu, s = to[:, :4], to[:, 4:12].reshape(B, 4, 2), to[:, 12:20].reshape(B, 4, 2)
    comp = torch.distributions.Independent(torch.distributions.Normal(mu, torch.exp(s)), 1)
    mix = torch.distributions.MixtureSameFamily(torch.distributions.Categorical(logits=logits), comp)
    (-mix.log_prob(torch.tensor(x)).mean()).backward()
    assert np.allclose(grad, to.grad.numpy(), rtol=1e-10, atol=1e-12)


def test_network_backward_against_autograd_and_differences():
    g = np.random.default_rng(3)
    params = Lr.init_params(4, 26)
    for k in ("b1", "b2", "b3"):
        params[k] = g.normal(size=params[k].shape) * 0.1
    X = Lr.standardise(g.normal(size=(6, 26)), np.zeros(26), np.ones(26))
    xt = g.normal(size=(6, 2))
    out, cache = Lr.forward(params, X)
    L, gout = Lr.mdn_nll_grad(out, xt)
    grads = Lr.backward(params, cache, gout)
    tp = {k: torch.tensor(v, requires_grad=True) for k, v in params.items()}
    tx = torch.tensor(X)
    gl = torch.nn.functional.gelu
    h1 = gl(tx @ tp["W1"].T + tp["b1"], approximate="tanh")
    h2 = gl(h1 @ tp["W2"].T + tp["b2"], approximate="tanh")
    o = h2 @ tp["W3"].T + tp["b3"]
    logits, mu, s = o[:, :4], o[:, 4:12].reshape(6, 4, 2), o[:, 12:20].reshape(6, 4, 2)
    comp = torch.distributions.Independent(torch.distributions.Normal(mu, torch.exp(s)), 1)
    mix = torch.distributions.MixtureSameFamily(torch.distributions.Categorical(logits=logits), comp)
    (-mix.log_prob(torch.tensor(xt)).mean()).backward()
    for k in params:
        assert np.allclose(grads[k], tp[k].grad.numpy(), rtol=1e-9, atol=1e-11), k
    h = 1e-6
    for k, idx in [("W1", (3, 5)), ("W2", (10, 200)), ("W3", (7, 99)), ("b1", (17,)), ("b3", (2,))]:
        pp, pm = {q: v.copy() for q, v in params.items()}, {q: v.copy() for q, v in params.items()}
        pp[k][idx] += h
        pm[k][idx] -= h
        fd = (Lr.mdn_nll_grad(Lr.forward(pp, X)[0], xt)[0] - Lr.mdn_nll_grad(Lr.forward(pm, X)[0], xt)[0]) / (2 * h)
        assert abs(fd - grads[k][idx]) < 1e-6 * max(1.0, abs(fd)), k


def test_adam_matches_torch():
    g = np.random.default_rng(5)
    params = {"a": g.normal(size=(3, 4)), "b": g.normal(size=5)}
    tp = [torch.tensor(params["a"].copy(), requires_grad=True), torch.tensor(params["b"].copy(), requires_grad=True)]
    opt = torch.optim.Adam(tp, lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    state = {}
    for t in range(1, 6):
        grads = {"a": g.normal(size=(3, 4)), "b": g.normal(size=5)}
        params = Lr.adam_step(params, grads, state, t, lr=1e-2)
        tp[0].grad = torch.tensor(grads["a"])
        tp[1].grad = torch.tensor(grads["b"])
        opt.step()
    assert np.allclose(params["a"], tp[0].detach().numpy(), rtol=1e-12)
    assert np.allclose(params["b"], tp[1].detach().numpy(), rtol=1e-12)


def test_mdn_sampling_law():
    g = np.random.default_rng(6)
    n = 20000
    row = _rand_out(g, 1)[0]
    out = np.broadcast_to(row, (n, Lr.D_OUT)).copy()
    xs, comp = Lr.mdn_sample(out, 77, 0, 3, np.arange(n))
    logits, mu, s = Lr.mdn_split(row[None])
    pi = np.exp(logits[0] - logits[0].max())
    pi /= pi.sum()
    assert np.allclose(np.bincount(comp, minlength=4) / n, pi, atol=0.015)
    for d in range(2):
        cdf = lambda v: np.sum(pi[None, :] * stats.norm.cdf((np.atleast_1d(v)[:, None] - mu[0, :, d]) / np.exp(s[0, :, d])), axis=1)
        assert stats.kstest(xs[:, d], cdf).pvalue > 1e-3


def _nonlin():
    spec = S.nonlin_c2(1)
    return spec, make_model(spec.kind, spec.dx, spec.dz, spec.dy, spec.blob)


def test_learned_step_with_transition_proposal_is_bootstrap_weight():
    """M = 1 and q = p(x_t | x_{t-1}) make the weight the likelihood of y_t."""
    spec, m = _nonlin()
    g = np.random.default_rng(7)
    N = 50
    st = {"x": g.normal(size=(N, 2)) * 2, "z": g.normal(size=(N, 1, 8)), "lam": np.zeros((N, 1)), "t": 3}
    out = np.zeros((N, Lr.D_OUT))
    out[:, 1:4] = -80.0                      # one live component
    gx = 0.5 * st["x"] + 25 * st["x"] / (1 + st["x"] ** 2)
    out[:, 4:6] = gx                         # its mean: the transition mean
    out[:, 12:14] = 0.0                      # log sd = log sqrt(qx) = 0
    y = g.normal(size=8)
    _, info = Lr.step(m, st, y, 9, 0, out, ess_frac=0.0)
    assert not info["fallback"]
    # with M = 1 the inner cloud is the single z; recompute z_t from the draws
    from oracle import philox as P
    zt = m.fz(st["x"], info["xt"], st["z"][:, 0], P.normals(9, 0, 4, np.arange(N), 0, P.NEW_Z, 8))
    assert np.allclose(info["logw"], m.logpy(y, info["xt"], zt), rtol=1e-10, atol=1e-10)


def test_learned_step_falls_back_to_lookahead_bit_for_bit():
    spec, m = _nonlin()
    _, _, ys = S.simulate(spec, 2, 3)
    st = ladpf.init_state(m, 40, 16, 5, 0)
    st, _ = ladpf.step(m, st, ys[0], 5, 0)
    out = np.zeros((40, Lr.D_OUT))
    out[:, 4:12] = 500.0                     # far from every particle
    out[:, 12:20] = math.log(1e-3)
    new, info = Lr.step(m, st, ys[1], 5, 0, out)
    assert info["fallback"]
    ref, _ = ladpf.step(m, st, ys[1], 5, 0)
    for k in ("x", "z", "lam"):
        assert np.array_equal(new[k], ref[k])


def test_features_are_cloud_moments():
    spec, m = _nonlin()
    st = ladpf.init_state(m, 10, 30, 1, 0)
    g = np.random.default_rng(8)
    lam = g.normal(size=(10, 30))
    st["lam"] = lam - np.log(np.exp(lam).sum(axis=1, keepdims=True))
    f = Lr.features(st, np.arange(8.0))
    q = np.exp(st["lam"][3])
    mean = (q[:, None] * st["z"][3]).sum(0)
    var = (q[:, None] * (st["z"][3] - mean) ** 2).sum(0)
    assert np.allclose(f[3], np.r_[st["x"][3], np.arange(8.0), mean, var])


@pytest.mark.parametrize("M", [4, 16])
def test_learned_weight_at_several_inner_particles(M):
    """M > 1, non-uniform inner weights, q = p(x_t | x_{t-1}) on a model whose
    f^x ignores z: eq:approx1 at x_t is the transition density itself (the
    inner weights sum to one), so the step-1 weight of Fig. 2 reduces to
    eq:approx2, log w = logsumexp_j log p(y | x_t, z_t^j) - log M.  Dropping
    the inner weights from eq:approx1, or the -log M of eq:approx2, shifts
    every weight by log M."""
    spec, m = _nonlin()
    g = np.random.default_rng(100 + M)
    N = 30
    lam = g.normal(size=(N, M)) * 1.5
    lam -= np.log(np.exp(lam).sum(axis=1, keepdims=True))
    st = {"x": g.normal(size=(N, 2)) * 2, "z": g.normal(size=(N, M, 8)), "lam": lam, "t": 3}
    out = np.zeros((N, Lr.D_OUT))
    out[:, 1:4] = -80.0                      # one live component
    gx = 0.5 * st["x"] + 25 * st["x"] / (1 + st["x"] ** 2)
    out[:, 4:6] = gx                         # the transition mean
    out[:, 12:14] = 0.0                      # log sd = log sqrt(qx) = 0
    y = g.normal(size=8)
    _, info = Lr.step(m, st, y, 9, 0, out, ess_frac=0.0)
    assert not info["fallback"]
    # eq:approx1 at x_t: the transition density (SciPy), whatever the inner weights
    ref_px = stats.norm.logpdf(info["xt"], gx, 1.0).sum(axis=1)
    assert np.allclose(info["log_px"], ref_px, rtol=1e-10, atol=1e-10)
    assert np.allclose(info["logq"], ref_px, rtol=1e-10, atol=1e-10)
    # the local resampling follows the inner weights: counts within floor/ceil of M qbar
    q = np.exp(lam)
    for i in range(N):
        cnt = np.bincount(info["binner"][i], minlength=M)
        assert np.all(cnt >= np.floor(M * q[i] - 1e-9)) and np.all(cnt <= np.ceil(M * q[i] + 1e-9))
    # z_t from the resampled components and the NEW_Z normals, then eq:approx2
    from oracle import philox as P
    ref = np.empty(N)
    for i in range(N):
        nu = P.normals(9, 0, 4, i, np.arange(M), P.NEW_Z, 8)
        zt = m.fz(st["x"][i], info["xt"][i], st["z"][i, info["binner"][i]], nu)
        ell = stats.norm.logpdf(y[None, :], zt + 0.05 * np.tile(info["xt"][i] ** 2, 4)[None, :],
                                np.sqrt(0.5)).sum(axis=1)
        ref[i] = np.log(np.mean(np.exp(ell - ell.max()))) + ell.max()
    assert np.allclose(info["logw"], ref, rtol=1e-10, atol=1e-9)
