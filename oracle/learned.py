"""Learned mixture-density proposal for the outer block, oracle side (FP64).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

The look-ahead DPF samples x_t from the Monte Carlo optimal proposal
eq:approx3.  A learned proposal q_phi(x_t | features) stands in for it: a
small network maps the features of an outer particle to a diagonal
Gaussian mixture over x_t, and the step that uses it is the importance
sampling step of Fig. 2 (step 1 weight) with pi = q_phi:

    log w_i = log p_Nz(y_t | xt_i, .)       (eq:approx2, unit inner weights)
            + log p_Nz(xt_i | x_{t-1}^{(i)}, .)  (eq:approx1, the inner mixture)
            - log q_phi(xt_i)

Features of outer particle i (raw, before standardisation):
    [x_{t-1}^{(i)} (dx), y_t (dy), sum_j qbar z (dz), sum_j qbar (z - mean)^2 (dz)].
Network: standardised features (padded to 32) -> 256 -> 256 -> 20 outputs, tanh
GELU (Hendrycks and Gimpel) after the two hidden layers.  Outputs: K = 4
mixture logits, K x dx means, K x dx log standard deviations clamped to
[log 1e-3, log 1e3].  Training minimises the mixture negative log-likelihood
of the x_t that the look-ahead DPF selects, with Adam (Kingma and Ba).

The network computes in BF16 on the GPU; ``forward(..., bf16=True)`` rounds
inputs, weights and hidden activations to BF16 (round to nearest even) and
does the arithmetic in FP64, so it predicts the GPU's values to within the
FP32 accumulation order.
"""
import math

import numpy as np

from . import philox as P
from .resample import (FLAG_DEGENERATE_INNER, FLAG_FALLBACK, logsumexp, normalise_log,
                       systematic_log, weights_from_log)
from . import ladpf

K_MIX = 4
D_IN = 32      # padded feature width
D_HID = 256
D_OUT = 20     # K (logits) + K*dx (means) + K*dx (log sds), dx = 2
LOG_SD_MIN = math.log(1e-3)
LOG_SD_MAX = math.log(1e3)
SQRT_2_OVER_PI = math.sqrt(2.0 / math.pi)


def bf16(a):
    """Round FP64 / FP32 values to the nearest BF16 value (ties to even)."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


def gelu(a):
    return 0.5 * a * (1.0 + np.tanh(SQRT_2_OVER_PI * (a + 0.044715 * a ** 3)))


def gelu_grad(a):
    u = SQRT_2_OVER_PI * (a + 0.044715 * a ** 3)
    th = np.tanh(u)
    du = SQRT_2_OVER_PI * (1.0 + 3.0 * 0.044715 * a * a)
    return 0.5 * (1.0 + th) + 0.5 * a * (1.0 - th * th) * du


def init_params(seed, d_feat):
    """He-style initialisation (FP64 masters); padded input columns are zero."""
    g = np.random.Generator(np.random.PCG64(seed))
    W1 = np.zeros((D_HID, D_IN))
    W1[:, :d_feat] = g.normal(0.0, math.sqrt(2.0 / d_feat), size=(D_HID, d_feat))
    W2 = g.normal(0.0, math.sqrt(2.0 / D_HID), size=(D_HID, D_HID))
    W3 = g.normal(0.0, 0.1 * math.sqrt(1.0 / D_HID), size=(D_OUT, D_HID))
    return {"W1": W1, "b1": np.zeros(D_HID), "W2": W2, "b2": np.zeros(D_HID),
            "W3": W3, "b3": np.zeros(D_OUT)}


def standardise(feat, mean, std):
    """(features - mean) / std, padded with zeros to D_IN columns."""
    f = (np.asarray(feat, dtype=np.float64) - mean) / std
    out = np.zeros(f.shape[:-1] + (D_IN,))
    out[..., :f.shape[-1]] = f
    return out


def forward(params, X, bf16_mode=False):
    """X (B, D_IN) standardised features -> (outputs (B, D_OUT), cache)."""
    q = bf16 if bf16_mode else (lambda v: v)
    W1, W2, W3 = q(params["W1"]), q(params["W2"]), q(params["W3"])
    x0 = q(X)
    a1 = x0 @ W1.T + params["b1"]
    h1 = q(gelu(a1))
    a2 = h1 @ W2.T + params["b2"]
    h2 = q(gelu(a2))
    out = h2 @ W3.T + params["b3"]
    return out, {"x0": x0, "a1": a1, "h1": h1, "a2": a2, "h2": h2}


def mdn_split(out, dx=2):
    K = K_MIX
    logits = out[..., :K]
    mu = out[..., K:K + K * dx].reshape(out.shape[:-1] + (K, dx))
    s_raw = out[..., K + K * dx:K + 2 * K * dx].reshape(out.shape[:-1] + (K, dx))
    return logits, mu, s_raw


def mdn_logpdf(out, x):
    """log q(x) of the diagonal mixture; out (..., D_OUT), x (..., dx)."""
    logits, mu, s_raw = mdn_split(out)
    s = np.clip(s_raw, LOG_SD_MIN, LOG_SD_MAX)
    logpi = logits - logsumexp(logits)[..., None]
    z = (x[..., None, :] - mu) / np.exp(s)
    lnorm = np.sum(-0.5 * z * z - s - 0.5 * math.log(2.0 * math.pi), axis=-1)
    return logsumexp(logpi + lnorm)


def mdn_nll_grad(out, x):
    """Mean negative log-likelihood over the batch and its gradient w.r.t. out."""
    B = out.shape[0]
    logits, mu, s_raw = mdn_split(out)
    s = np.clip(s_raw, LOG_SD_MIN, LOG_SD_MAX)
    inside = (s_raw > LOG_SD_MIN) & (s_raw < LOG_SD_MAX)
    lse_l = logsumexp(logits)
    logpi = logits - lse_l[:, None]
    sd = np.exp(s)
    z = (x[:, None, :] - mu) / sd
    lnorm = np.sum(-0.5 * z * z - s - 0.5 * math.log(2.0 * math.pi), axis=-1)
    ell = logpi + lnorm
    L = logsumexp(ell)
    gam = np.exp(ell - L[:, None])
    pi = np.exp(logpi)
    g_logits = pi - gam
    g_mu = -gam[:, :, None] * z / sd
    g_s = -gam[:, :, None] * (z * z - 1.0) * inside
    grad = np.concatenate([g_logits, g_mu.reshape(B, -1), g_s.reshape(B, -1)], axis=1) / B
    return float(np.mean(-L)), grad


def backward(params, cache, g_out):
    """Gradients of all parameters from d loss / d outputs (FP64)."""
    h2, a2, h1, a1, x0 = cache["h2"], cache["a2"], cache["h1"], cache["a1"], cache["x0"]
    grads = {"W3": g_out.T @ h2, "b3": g_out.sum(axis=0)}
    d_a2 = (g_out @ params["W3"]) * gelu_grad(a2)
    grads["W2"] = d_a2.T @ h1
    grads["b2"] = d_a2.sum(axis=0)
    d_a1 = (d_a2 @ params["W2"]) * gelu_grad(a1)
    grads["W1"] = d_a1.T @ x0
    grads["b1"] = d_a1.sum(axis=0)
    return grads


def adam_step(params, grads, state, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t starts at 1); state holds m and v per parameter."""
    for k in params:
        m = state.setdefault("m_" + k, np.zeros_like(params[k]))
        v = state.setdefault("v_" + k, np.zeros_like(params[k]))
        m[...] = b1 * m + (1.0 - b1) * grads[k]
        v[...] = b2 * v + (1.0 - b2) * grads[k] ** 2
        mh = m / (1.0 - b1 ** t)
        vh = v / (1.0 - b2 ** t)
        params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
    return params


def features(state, y):
    """Raw features of every outer particle of a look-ahead state."""
    m, v = ladpf.cloud_moments(state["z"], state["lam"])
    N = state["x"].shape[0]
    yy = np.broadcast_to(np.asarray(y, dtype=np.float64), (N, len(y)))
    return np.concatenate([state["x"], yy, m, v], axis=1)


def mdn_sample(out, seed, fid, t, i):
    """Draw from the mixture of each row: component by U53 (MDN_U at (t, i, 0))
    over softmax(logits), then mu + sd * normals (MDN_X at (t, i, 0))."""
    logits, mu, s_raw = mdn_split(out)
    s = np.clip(s_raw, LOG_SD_MIN, LOG_SD_MAX)
    n = out.shape[0]
    u = P.uniform53(seed, fid, t, i, P.MDN_U)
    comp = np.empty(n, dtype=np.int64)
    for r in range(n):
        c, _, _ = systematic_log(logits[r], 1, float(u[r]))
        comp[r] = c[0]
    nu = P.normals(seed, fid, t, i, 0, P.MDN_X, mu.shape[-1])
    rows = np.arange(n)
    x = mu[rows, comp] + np.exp(s[rows, comp]) * nu
    return x, comp


def step(model, state, y, seed, fid, mdn_out, ess_frac=0.1):
    """One step with the learned proposal, falling back to the look-ahead step.

    mdn_out: network outputs (N, D_OUT) for the current state's particles.
    Returns (new_state, info); info["fallback"] says which path was taken.
    """
    x, z, lam = state["x"], state["z"], state["lam"]
    t = state["t"] + 1
    N, M = lam.shape
    xt, comp = mdn_sample(mdn_out, seed, fid, t, np.arange(N))
    logq = mdn_logpdf(mdn_out, xt)
    zt = np.empty_like(z)
    lt = np.empty_like(lam)
    log_px = np.empty(N)
    log_py = np.empty(N)
    binner = np.empty((N, M), dtype=np.int64)
    u_in = P.uniform53(seed, fid, t, np.arange(N), P.INNER_U)
    j = np.arange(M)
    flags = 0
    for i in range(N):
        kappa = lam[i] + model.logpx(xt[i], x[i], z[i], t - 1)
        log_px[i] = logsumexp(kappa)                       # eq:approx1 at xt_i
        b, deg_i, _ = systematic_log(kappa, M, float(u_in[i]))
        if deg_i:
            flags |= FLAG_DEGENERATE_INNER
        binner[i] = b
        nu = P.normals(seed, fid, t, i, j, P.NEW_Z, model.dz)
        zt[i] = model.fz(x[i], xt[i], z[i, b], nu, t - 1)
        ell = model.logpy(y, xt[i], zt[i])
        log_py[i] = logsumexp(ell) - math.log(M)           # eq:approx2, unit weights
        lt[i], _ = normalise_log(ell)
    logw = log_py + log_px - logq
    Wn, deg, _ = weights_from_log(logw)
    Wbar = Wn / Wn.sum()
    ess = 1.0 / np.sum(Wbar ** 2)
    info = {"xt": xt, "comp": comp, "logq": logq, "log_px": log_px, "log_py": log_py,
            "logw": logw, "ess": ess, "binner": binner}
    if deg or ess < ess_frac * N:
        new_state, la_info = ladpf.step(model, state, y, seed, fid)
        info.update(la_info)
        info["fallback"] = True
        info["flags"] = la_info["flags"] | FLAG_FALLBACK
        return new_state, info
    u = float(P.uniform53(seed, fid, t, 0, P.OUTER_U))
    A, _, _ = systematic_log(logw, N, u)
    new_state = {"x": xt[A], "z": zt[A], "lam": lt[A], "t": t}
    info.update({"A": A, "fallback": False, "flags": flags,
                 "xhat": xt[A].mean(axis=0),
                 "zhat": np.einsum("nm,nmd->d", np.exp(lt[A]), zt[A]) / N,
                 "dlogz": logsumexp(logw) - math.log(N)})
    return new_state, info
