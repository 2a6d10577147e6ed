"""One time step of the look-ahead DPF (Section 2.2, Fig. 4), FP64.

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

State after step t-1 of one filter: outer particles x_{t-1}^{(i)} (N, dx),
inner clouds z_{t-1}^{(i,j)} (N, M, dz) and the normalised inner
log-weights lam^{(i,j)} = log qbar_{t-1}^{(i,j)} (N, M) of eq:qbar.  The
outer particles are equally weighted (each step ends with outer resampling).

Step t, given y_t, in the order of Fig. 4:

1. Look-ahead particles.  For every outer i and every inner j, one
   candidate xla^{(i,j)} ~ p(x_t | x_{t-1}^{(i)}, z_{t-1}^{(i,j)}) and its
   companion zla^{(i,j)} ~ p(z_t | x_{t-1}^{(i)}, xla^{(i,j)}, z_{t-1}^{(i,j)}).
   Drawing x from every inner component once, weighted by qbar, is the
   mixture eq:approx1; each candidate carries one companion z
   (N_x' = M candidates with N_z' = 1 companion each, the O(N M) cost stated
   after eq:weightsMC).  Both come from one draw at (t, i, j) of purpose
   LA_X: normals 0 .. dx-1 for x, dx .. dx+dz-1 for z (packed layout).
2. Weights (eq:weightsMC): ell^{(i,j)} = lam^{(i,j)} + log p(y_t | xla, zla)
   and log w^{(i)} = logsumexp_j ell^{(i,j)}, an estimate of the predictive
   likelihood p(y_t | y_{0:t-1}, x_{0:t-1}^{(i)}) that eq:weightsopt makes the
   optimal-proposal weight.
3. Outer resampling at t-1 with those weights (systematic, U53 OUTER_U).
4. New particles.  For new particle k with parent p = A_k:
   x_t^{(k)} is drawn from the MC optimal proposal eq:approx3 by
   sampling-importance-resampling over the parent's M candidates with
   probabilities proportional to exp(ell^{(p,j)}) (U53 CAND_U);
   the parent's cloud is conditioned on x_t^{(k)} as in eq:qnobar,
   kappa^{(j)} = lam^{(p,j)} + log p(x_t^{(k)} | x_{t-1}^{(p)}, z_{t-1}^{(p,j)}),
   resampled systematically (U53 INNER_U), and propagated with the prior
   inner proposal (the inner predictive of Section 2, importance weight 1):
   z_t^{(k,j)} ~ p(z_t | x_{t-1}^{(p)}, x_t^{(k)}, z_{t-1}^{(p,b_j)}) (NEW_Z);
   finally the inner measurement update eq:qbar gives
   lam_t^{(k,j)} = log p(y_t | x_t^{(k)}, z_t^{(k,j)}) - logsumexp_j(.).

Nested look-ahead estimator (optional, n_comp = K >= 1).  Fig. 4 step 1
draws N_x' candidates and, for each, N_z' companions from the inner
predictive given that candidate; eq:weightsMC averages p(y_t | .) over all
of them.  With K companions per candidate (N_x' = M stratified candidates as
above, N_z' = K): the companions of candidate xla^{(i,m)} take ancestors
b_1..b_K by systematic resampling (U53 LA_B at (t, i, m)) of the inner
weights conditioned on the candidate as in eq:qnobar,
kappa_j = lam^{(i,j)} + log p(xla^{(i,m)} | x_{t-1}^{(i)}, z_{t-1}^{(i,j)}),
and are propagated with the inner prior, zla^{(i,m,k)} ~
p(z_t | x_{t-1}^{(i)}, xla^{(i,m)}, z_{t-1}^{(i,b_k)}) (LA_Z normals k dz ..
k dz + dz - 1 of the draw at (t, i, m), block-aligned layout); then
ell^{(i,m)} = lam^{(i,m)} + log (1/K) sum_k p(y_t | xla^{(i,m)}, zla^{(i,m,k)})
and log w^{(i)} = logsumexp_m ell^{(i,m)} as before.  Steps 3-4 are
unchanged (the SIR of step 4 uses these ell).  Cost K M^2 model
evaluations per outer particle where p(x_t | x_{t-1}, z_{t-1}) depends on z,
K M otherwise (kappa is then lam up to a constant).

Predicted observation (models with a noise-free observation mean h): the
look-ahead draws are draws from the one-step predictive p(x_t, z_t | y_{0:t-1})
with weights qbar^{(i,j)} / N, so yhat_{t|t-1} = (1/N) sum_i sum_j
qbar^{(i,j)} h(xla^{(i,j)}, zla^{(i,j)}) (nested: the mean over each
candidate's companions).  Its error y_t - yhat is the reward signal of the
decomposition choice of Section 3.

Estimates: xhat = mean_k x_t^{(k)}, zhat = mean_k sum_j qbar_t z_t,
ESS of the look-ahead weights, dlogZ = logsumexp_i log w - log N, and the
Rao-Blackwellised xhat_rb = sum_i Wbar_i sum_j pi_ij xla^{(i,j)} (the exact
conditional expectation of the new x given the look-ahead draws).
"""
import math

import numpy as np

from . import philox as P
from .resample import (FLAG_DEGENERATE_INNER, FLAG_DEGENERATE_OUTER, FLAG_NONFINITE,
                       logsumexp, normalise_log, systematic_log, weights_from_log)


def init_state(model, N, M, seed, fid):
    """Prior draws [x_0; z_0] ~ N(0, I) and lam_0 = -log M."""
    i = np.arange(N)
    j = np.arange(M)
    x0 = P.normals(seed, fid, 0, i, 0, P.INIT_X, model.dx)
    z0 = P.normals(seed, fid, 0, i[:, None], j[None, :], P.INIT_Z, model.dz)
    lam0 = np.full((N, M), -math.log(M))
    return {"x": x0, "z": z0, "lam": lam0, "t": 0}


def cloud_moments(z, lam):
    """qbar-weighted mean and variance of each inner cloud, (N, dz) each."""
    q = np.exp(lam)
    m = np.einsum("nm,nmd->nd", q, z)
    v = np.einsum("nm,nmd->nd", q, (z - m[:, None, :]) ** 2)
    return m, v


def lookahead(model, state, y, seed, fid, rows=None):
    """Fig. 4 steps 1-2 for all outer particles; returns (xla, zla, ell, logw).
    rows: the outer indices of the state's rows (their random-number
    counters), by default 0 .. N-1; a subset of a filter's particles gives
    exactly those particles' values."""
    x, z, lam = state["x"], state["z"], state["lam"]
    t = state["t"] + 1
    N, M = lam.shape
    i = (np.arange(N) if rows is None else np.asarray(rows))[:, None]
    j = np.arange(M)[None, :]
    # one draw per candidate: x first, then z
    nu = P.normals(seed, fid, t, i, j, P.LA_X, model.dx + model.dz)
    nu_x, nu_z = nu[..., :model.dx], nu[..., model.dx:]
    xp = x[:, None, :]
    xla = model.fx(xp, z, nu_x, t - 1)
    zla = model.fz(xp, xla, z, nu_z, t - 1)
    ell = lam + model.logpy(y, xla, zla)
    logw = logsumexp(ell)
    return xla, zla, ell, logw


def lookahead_nested(model, state, y, seed, fid, K, u_comp=None):
    """Fig. 4 steps 1-2 with K companions per candidate (the nested estimator
    of eq:weightsMC, see the module text); returns (xla, ell, logw, comp),
    comp[i, m] the K companion ancestors of candidate (i, m).  u_comp
    replaces the LA_B offsets (test hook)."""
    x, z, lam = state["x"], state["z"], state["lam"]
    t = state["t"] + 1
    N, M = lam.shape
    dz = model.dz
    i_ = np.arange(N)[:, None]
    j_ = np.arange(M)[None, :]
    nu_x = P.normals(seed, fid, t, i_, j_, P.LA_X, model.dx)
    xla = model.fx(x[:, None, :], z, nu_x, t - 1)
    nu_z = P.normals_blocked(seed, fid, t, i_, j_, P.LA_Z, K * dz).reshape(N, M, K, dz)
    if u_comp is None:
        u_comp = P.uniform53_ab(seed, fid, t, i_, j_, P.LA_B)
    ell = np.empty((N, M))
    comp = np.empty((N, M, K), dtype=np.int64)
    hmean = np.zeros((N, M, model.dy)) if hasattr(model, "obs_mean") else None
    for i in range(N):
        for m in range(M):
            # inner weights conditioned on the candidate (eq:qnobar)
            kappa = lam[i] + model.logpx(xla[i, m], x[i], z[i], t - 1)
            b, _, _ = systematic_log(kappa, K, float(u_comp[i, m]))
            comp[i, m] = b
            zc = model.fz(x[i], xla[i, m], z[i, b], nu_z[i, m], t - 1)
            ell[i, m] = lam[i, m] + logsumexp(model.logpy(y, xla[i, m], zc)) - math.log(K)
            if hmean is not None:
                hmean[i, m] = np.mean(model.obs_mean(xla[i, m], zc), axis=0)
    logw = logsumexp(ell)
    return xla, ell, logw, comp, hmean


def predicted_observation(lam, hmean):
    """yhat_{t|t-1} = (1/N) sum_i sum_j qbar^{(i,j)} h^{(i,j)}: the look-ahead
    draws weighted as draws from the one-step predictive."""
    N = lam.shape[0]
    return np.einsum("nm,nmd->d", np.exp(lam), hmean) / N


def step(model, state, y, seed, fid, u_outer=None, u_cand=None, u_inner=None, n_comp=0, ell_given=None):
    """One look-ahead DPF step consuming y_t.  Returns (new_state, info).

    The ``u_*`` arguments replace the Philox offsets (test hooks for
    enumerating resampling outcomes); by default they come from the
    random-number contract.  n_comp >= 1: the nested look-ahead estimator
    with that many companions per candidate; 0: one companion drawn with
    the candidate from the same inner component.  ell_given (N, M): take
    these look-ahead log-weights instead of computing them (test hook for
    checking steps 3-4 on given weights); the candidates are still drawn.
    """
    x, z, lam = state["x"], state["z"], state["lam"]
    t = state["t"] + 1
    N, M = lam.shape
    flags = 0

    comp = None
    yhat = None
    if n_comp:
        xla, ell, logw, comp, hmean = lookahead_nested(model, state, y, seed, fid, n_comp)
        zla = None
    else:
        xla, zla, ell, logw = lookahead(model, state, y, seed, fid)
        hmean = model.obs_mean(xla, zla) if hasattr(model, "obs_mean") else None
    if hmean is not None:
        yhat = predicted_observation(lam, hmean)
    if ell_given is not None:
        ell = np.asarray(ell_given, dtype=np.float64)
        logw = logsumexp(ell)

    # Step 3: outer resampling with the look-ahead weights.
    if u_outer is None:
        u_outer = float(P.uniform53(seed, fid, t, 0, P.OUTER_U))
    A, deg, nonf = systematic_log(logw, N, u_outer)
    if deg:
        flags |= FLAG_DEGENERATE_OUTER
    if nonf:
        flags |= FLAG_NONFINITE
    Wn, _, _ = weights_from_log(logw)
    Wbar = Wn / np.sum(Wn)
    ess = 1.0 / np.sum(Wbar ** 2)
    lse_all = logsumexp(logw)
    dlogz = lse_all - math.log(N)

    # Rao-Blackwellised estimate of the new x.
    pi = np.stack([weights_from_log(ell[i])[0] for i in range(N)])
    pi = pi / pi.sum(axis=1, keepdims=True)
    xhat_rb = np.einsum("n,nm,nmd->d", Wbar, pi, xla)

    # Step 4: new particles.
    if u_cand is None:
        u_cand = P.uniform53(seed, fid, t, np.arange(N), P.CAND_U)
    if u_inner is None:
        u_inner = P.uniform53(seed, fid, t, np.arange(N), P.INNER_U)
    xnew = np.empty_like(x)
    znew = np.empty_like(z)
    lamnew = np.empty_like(lam)
    cand = np.empty(N, dtype=np.int64)
    binner = np.empty((N, M), dtype=np.int64)
    for k in range(N):
        p = A[k]
        xnew[k], znew[k], lamnew[k], cand[k], binner[k], fl = new_particle(
            model, x[p], z[p], lam[p], ell[p], xla[p], y, seed, fid, t, k, float(u_cand[k]), float(u_inner[k]))
        flags |= fl

    xhat = xnew.mean(axis=0)
    zhat = np.einsum("nm,nmd->d", np.exp(lamnew), znew) / N
    new_state = {"x": xnew, "z": znew, "lam": lamnew, "t": t}
    info = {
        "xla": xla, "zla": zla, "comp": comp, "ell": ell, "logw": logw, "A": A, "cand": cand,
        "binner": binner, "u_outer": u_outer, "u_cand": np.asarray(u_cand),
        "u_inner": np.asarray(u_inner),
        "xhat": xhat, "zhat": zhat, "ess": ess, "dlogz": dlogz, "xhat_rb": xhat_rb,
        "yhat": yhat, "flags": flags,
    }
    return new_state, info


def new_particle(model, xp, zp, lamp, ellp, xlap, y, seed, fid, t, k, u_cand_k, u_inner_k):
    """Fig. 4 step 4 for new particle k whose parent p has x xp (dx,), cloud
    zp (M, dz), inner log-weights lamp (M,), look-ahead log-weights ellp
    (M,) and candidates xlap (M, dx): the candidate by SIR over ellp (U53
    u_cand_k), the cloud conditioned on it (eq:qnobar) and resampled
    systematically (u_inner_k), propagated (NEW_Z at (t, k, j)) and updated
    (eq:qbar).  Returns (x_t, z_t (M, dz), lam_t (M,), candidate, inner
    ancestors (M,), flags)."""
    M = lamp.shape[0]
    flags = 0
    c, _, _ = systematic_log(ellp, 1, u_cand_k)
    xk = xlap[c[0]]
    kappa = lamp + model.logpx(xk, xp, zp, t - 1)
    b, deg_i, nonf_i = systematic_log(kappa, M, u_inner_k)
    if deg_i:
        flags |= FLAG_DEGENERATE_INNER
    if nonf_i:
        flags |= FLAG_NONFINITE
    nu = P.normals(seed, fid, t, k, np.arange(M), P.NEW_Z, model.dz)
    zk = model.fz(xp, xk, zp[b], nu, t - 1)
    lamk, deg_l = normalise_log(model.logpy(y, xk, zk))
    if deg_l:
        flags |= FLAG_DEGENERATE_INNER
    return xk, zk, lamk, int(c[0]), b, flags


def training_pairs(state, y, info):
    """(features of the parent, SIR-selected x_t) for every new particle.

    Features: [x_{t-1}^{(p)}, y_t, qbar-weighted mean and variance of the
    parent's cloud] -- the inputs the learned proposal conditions on.
    """
    m, v = cloud_moments(state["z"], state["lam"])
    A = info["A"]
    N = len(A)
    yy = np.broadcast_to(np.asarray(y, dtype=np.float64), (N, len(y)))
    feats = np.concatenate([state["x"][A], yy, m[A], v[A]], axis=1)
    return feats, state_x_new(info)


def state_x_new(info):
    A, cand, xla = info["A"], info["cand"], info["xla"]
    return xla[A, cand]


def run(model, N, M, ys, seed, fid, n_comp=0):
    """Run the look-ahead DPF over observations y_1..y_T; returns per-step estimates."""
    state = init_state(model, N, M, seed, fid)
    out = {"xhat": [], "zhat": [], "ess": [], "dlogz": [], "xhat_rb": [], "flags": 0}
    for y in ys:
        state, info = step(model, state, y, seed, fid, n_comp=n_comp)
        for key in ("xhat", "zhat", "ess", "dlogz", "xhat_rb"):
            out[key].append(info[key])
        out["flags"] |= info["flags"]
    for key in ("xhat", "zhat", "ess", "dlogz", "xhat_rb"):
        out[key] = np.asarray(out[key])
    out["state"] = state
    return out
