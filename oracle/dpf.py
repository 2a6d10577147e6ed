"""One time step of the plain DPF (Section 2, Fig. 2) with prior proposals, FP64.

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

With the prior proposals of Section 2.1 (the x proposal is the MC predictive
eq:approx1 and the z proposal the inner predictive), the ratio in the
step-1 weight of Fig. 2 is one and the inner importance weight r-tilde is
one, so the DPF state between steps is the proposed pair
(xt^{(i)}, zt^{(i,j)}) for the next time, equally weighted.

Step t, given y_t (Fig. 2):
 1. ell^{(i,j)} = log p(y_t | xt^{(i)}, zt^{(i,j)});
    log w^{(i)} = logsumexp_j ell - log M        (eq:approx2 with r-tilde = 1)
    Estimates use Wbar = softmax(log w) and qbar = softmax_j ell (step 3
    weights, eq:qbar): xhat = sum_i Wbar_i xt_i,
    zhat = sum_i Wbar_i sum_j qbar_ij zt_ij,  dlogZ = logsumexp_i log w - log N.
 2. Outer systematic resampling with w (U53 OUTER_U).
 3. Inner measurement update qbar (already formed above).
 4-7. ``propose``: for new particle k with parent p = A_k
    a_k ~ Cat(qbar_p) (U53 DPF_ANC_U) and xt_{t+1}^{(k)} ~ p(x | xt_p, zt_{p,a_k})
    -- a draw from the mixture eq:approx1 (DPF_X normals);
    kappa_j = log qbar_pj + log p(xt_{t+1}^{(k)} | xt_p, zt_pj)  (eq:qnobar);
    inner systematic resampling with kappa (U53 INNER_U);
    zt_{t+1}^{(k,j)} ~ p(z | xt_p, xt_{t+1}^{(k)}, zt_{p,b_j})  (DPF_Z normals).
Initialisation draws the prior (INIT_X, INIT_Z) and runs steps 4-7 at t = 0
with every parent its own ancestor and uniform qbar (no y_0 is consumed).
"""
import math

import numpy as np

from . import philox as P
from .resample import (FLAG_DEGENERATE_INNER, FLAG_DEGENERATE_OUTER, FLAG_NONFINITE,
                       logsumexp, normalise_log, systematic_log, weights_from_log)


def propose(model, x, z, lq, A, t, seed, fid):
    """Fig. 2 steps 4-7 at time t: returns (xt_{t+1}, zt_{t+1}, anc, binner, flags)."""
    N = len(A)
    M = z.shape[1]
    flags = 0
    u_anc = P.uniform53(seed, fid, t, np.arange(N), P.DPF_ANC_U)
    u_inner = P.uniform53(seed, fid, t, np.arange(N), P.INNER_U)
    nu_x = P.normals(seed, fid, t, np.arange(N), 0, P.DPF_X, model.dx)
    xn = np.empty((N, model.dx))
    zn = np.empty((N, M, model.dz))
    anc = np.empty(N, dtype=np.int64)
    binner = np.empty((N, M), dtype=np.int64)
    j = np.arange(M)
    for k in range(N):
        p = A[k]
        a, _, _ = systematic_log(lq[p], 1, float(u_anc[k]))
        anc[k] = a[0]
        xn[k] = model.fx(x[p], z[p, anc[k]], nu_x[k], t)
        kappa = lq[p] + model.logpx(xn[k], x[p], z[p], t)
        b, deg_i, nonf_i = systematic_log(kappa, M, float(u_inner[k]))
        if deg_i:
            flags |= FLAG_DEGENERATE_INNER
        if nonf_i:
            flags |= FLAG_NONFINITE
        binner[k] = b
        nu = P.normals(seed, fid, t, k, j, P.DPF_Z, model.dz)
        zn[k] = model.fz(x[p], xn[k], z[p, b], nu, t)
    return xn, zn, anc, binner, flags


def init_state(model, N, M, seed, fid):
    i = np.arange(N)
    j = np.arange(M)
    x0 = P.normals(seed, fid, 0, i, 0, P.INIT_X, model.dx)
    z0 = P.normals(seed, fid, 0, i[:, None], j[None, :], P.INIT_Z, model.dz)
    lq0 = np.full((N, M), -math.log(M))
    xt, zt, _, _, flags = propose(model, x0, z0, lq0, np.arange(N), 0, seed, fid)
    return {"xt": xt, "zt": zt, "t": 0, "flags": flags}


def step(model, state, y, seed, fid):
    """One plain DPF step consuming y_t; returns (new_state, info)."""
    xt, zt = state["xt"], state["zt"]
    t = state["t"] + 1
    N, M = zt.shape[0], zt.shape[1]
    flags = 0

    ell = model.logpy(y, xt[:, None, :], zt)
    logw = logsumexp(ell) - math.log(M)
    lq, deg_rows = normalise_log(ell)
    if deg_rows.any():
        flags |= FLAG_DEGENERATE_INNER

    Wn, _, _ = weights_from_log(logw)
    Wbar = Wn / np.sum(Wn)
    ess = 1.0 / np.sum(Wbar ** 2)
    dlogz = logsumexp(logw) - math.log(N)
    xhat = Wbar @ xt
    zhat = np.einsum("n,nm,nmd->d", Wbar, np.exp(lq), zt)

    u = float(P.uniform53(seed, fid, t, 0, P.OUTER_U))
    A, deg, nonf = systematic_log(logw, N, u)
    if deg:
        flags |= FLAG_DEGENERATE_OUTER
    if nonf:
        flags |= FLAG_NONFINITE

    xn, zn, anc, binner, f2 = propose(model, xt, zt, lq, A, t, seed, fid)
    flags |= f2
    new_state = {"xt": xn, "zt": zn, "t": t, "flags": 0}
    info = {"ell": ell, "logw": logw, "A": A, "anc": anc, "binner": binner,
            "xhat": xhat, "zhat": zhat, "ess": ess, "dlogz": dlogz, "flags": flags}
    return new_state, info


def run(model, N, M, ys, seed, fid):
    state = init_state(model, N, M, seed, fid)
    out = {"xhat": [], "zhat": [], "ess": [], "dlogz": [], "flags": state["flags"]}
    for y in ys:
        state, info = step(model, state, y, seed, fid)
        for key in ("xhat", "zhat", "ess", "dlogz"):
            out[key].append(info[key])
        out["flags"] |= info["flags"]
    for key in ("xhat", "zhat", "ess", "dlogz"):
        out[key] = np.asarray(out[key])
    out["state"] = state
    return out
