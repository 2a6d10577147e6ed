"""Step-level comparison of the HIP path with the FP64 oracle.

Both sides start from the same FP32 state and the same Philox streams.  The
GPU computes in FP32, the oracle in FP64, so a resampling index may flip
where a systematic point lies within the FP32 error of a cumulative-weight
boundary.  Such flips are legitimate (both answers are correct draws); every
index mismatch must be explained by a near tie in the oracle's own
cumulative weights, and values are compared only where all upstream indices
agree.

Tolerances (derived from the arithmetic):
  * log-weights: |d| <= 1e-4 * max(1, |ref|)    (FP32 sums of O(10) terms)
  * states:      |d| <= 1e-4 * max(1, |ref|)    (the 1e-4 relative target)
  * near tie:    a point within DELTA * C_total of a boundary, DELTA = 1e-4
"""
import math

import numpy as np

from oracle import ladpf, dpf
from oracle import philox as P
from oracle.resample import normalise_log, weights_from_log

TOL = 1e-4
DELTA = 1e-4


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    both_inf = np.isinf(a) & np.isinf(b) & (np.sign(a) == np.sign(b))
    d = np.where(both_inf, 0.0, np.abs(a - b) / np.maximum(1.0, np.abs(b)))
    return float(np.max(d)) if d.size else 0.0


def near_tie(w, u, n_out, k, a, b, delta=DELTA):
    """True if systematic point k lies within delta*total of every boundary
    separating indices a and b of weights w (FP64)."""
    C = np.cumsum(np.asarray(w, dtype=np.float64))
    tot = C[-1]
    pt = ((k + u) * tot) / n_out
    lo, hi = min(a, b), max(a, b)
    return bool(np.all(np.abs(C[lo:hi] - pt) <= delta * tot))


def to_state32(state):
    """Round an oracle state to FP32 (both sides start from these values)."""
    out = dict(state)
    for key in ("x", "z", "lam", "xt", "zt"):
        if key in out:
            out[key] = np.asarray(out[key], dtype=np.float32).astype(np.float64)
    return out


class Report(dict):
    def line(self):
        return ", ".join("%s=%s" % (k, ("%.3g" % v) if isinstance(v, float) else v) for k, v in self.items())


def compare_la(model, st32, y32, seed, fid, g_state, g_ell, g_logw, g_anc, g_sel, **step_kw):
    """Compare one look-ahead step.  g_* are the GPU's results as numpy
    arrays in oracle layout; step_kw go to the oracle's step.  Returns
    (report, oracle_new_state, info)."""
    new_o, info = ladpf.step(model, st32, y32, seed, fid, **step_kw)
    N, M = st32["lam"].shape
    r = Report()
    r["err_ell"] = rel_err(g_ell, info["ell"])
    r["err_logw"] = rel_err(g_logw, info["logw"])
    w_out, _, _ = weights_from_log(info["logw"])
    A_o, A_g = info["A"], g_anc
    bad_anc = np.nonzero(A_o != A_g)[0]
    r["anc_flips"] = len(bad_anc)
    r["anc_unexplained"] = sum(not near_tie(w_out, info["u_outer"], N, k, A_o[k], A_g[k]) for k in bad_anc)
    ok = A_o == A_g
    bad_sel = np.nonzero(ok & (g_sel != info["cand"]))[0]
    r["cand_flips"] = len(bad_sel)
    unexpl = 0
    for k in bad_sel:
        p = A_o[k]
        wc, _, _ = weights_from_log(info["ell"][p])
        unexpl += not near_tie(wc, info["u_cand"][k], 1, 0, info["cand"][k], g_sel[k])
    r["cand_unexplained"] = unexpl
    good = ok & (g_sel == info["cand"])
    r["err_x"] = rel_err(g_state["x"][good], new_o["x"][good])
    # inner clouds: per (k, j) the resampled ancestor may flip at a near tie
    zg, zo = g_state["z"], new_o["z"]
    dz = np.max(np.abs(zg - zo) / np.maximum(1.0, np.abs(zo)), axis=2)  # (N, M)
    zflip = good[:, None] & (dz > TOL)
    r["z_flips"] = int(zflip.sum())
    unexpl = 0
    for k, j in zip(*np.nonzero(zflip)):
        p = A_o[k]
        kap = st32["lam"][p] + model.logpx(new_o["x"][k], st32["x"][p], st32["z"][p], st32["t"])
        wk, _, _ = weights_from_log(kap)
        b = info["binner"][k, j]
        C = np.cumsum(wk)
        Pj = ((j + info["u_inner"][k]) * C[-1]) / M
        near = abs(Pj - C[b]) <= DELTA * C[-1] or (b > 0 and abs(Pj - C[b - 1]) <= DELTA * C[-1])
        unexpl += not near
    r["z_unexplained"] = unexpl
    clean = good & ~zflip.any(axis=1)
    r["err_z"] = rel_err(zg[clean], zo[clean])
    r["err_lam"] = rel_err(g_state["lam"][clean], new_o["lam"][clean])
    r["clean_frac"] = float(clean.mean())
    return r, new_o, info


def compare_plain(model, st32, y32, seed, fid, g_state, g_ell, g_logw, g_anc, g_sel):
    """Compare one plain DPF step (state = proposals xt, zt)."""
    new_o, info = dpf.step(model, st32, y32, seed, fid)
    N = st32["xt"].shape[0]
    M = st32["zt"].shape[1]
    r = Report()
    r["err_ell"] = rel_err(g_ell, info["ell"])
    r["err_logw"] = rel_err(g_logw, info["logw"])
    w_out, _, _ = weights_from_log(info["logw"])
    u_out = float(P.uniform53(seed, fid, st32["t"] + 1, 0, P.OUTER_U))
    A_o, A_g = info["A"], g_anc
    bad_anc = np.nonzero(A_o != A_g)[0]
    r["anc_flips"] = len(bad_anc)
    r["anc_unexplained"] = sum(not near_tie(w_out, u_out, N, k, A_o[k], A_g[k]) for k in bad_anc)
    ok = A_o == A_g
    t = st32["t"] + 1
    u_anc = P.uniform53(seed, fid, t, np.arange(N), P.DPF_ANC_U)
    u_in = P.uniform53(seed, fid, t, np.arange(N), P.INNER_U)
    bad_sel = np.nonzero(ok & (g_sel != info["anc"]))[0]
    r["sel_flips"] = len(bad_sel)
    unexpl = 0
    for k in bad_sel:
        wq, _, _ = weights_from_log(info["ell"][A_o[k]])
        unexpl += not near_tie(wq, u_anc[k], 1, 0, info["anc"][k], g_sel[k])
    r["sel_unexplained"] = unexpl
    good = ok & (g_sel == info["anc"])
    r["err_x"] = rel_err(g_state["x"][good], new_o["xt"][good])
    zg, zo = g_state["z"], new_o["zt"]
    dz = np.max(np.abs(zg - zo) / np.maximum(1.0, np.abs(zo)), axis=2)
    zflip = good[:, None] & (dz > TOL)
    r["z_flips"] = int(zflip.sum())
    lq, _ = normalise_log(info["ell"])
    unexpl = 0
    for k, j in zip(*np.nonzero(zflip)):
        p = A_o[k]
        kap = lq[p] + model.logpx(new_o["xt"][k], st32["xt"][p], st32["zt"][p], st32["t"] + 1)
        wk, _, _ = weights_from_log(kap)
        b = info["binner"][k, j]
        C = np.cumsum(wk)
        Pj = ((j + u_in[k]) * C[-1]) / M
        near = abs(Pj - C[b]) <= DELTA * C[-1] or (b > 0 and abs(Pj - C[b - 1]) <= DELTA * C[-1])
        unexpl += not near
    r["z_unexplained"] = unexpl
    clean = good & ~zflip.any(axis=1)
    r["err_z"] = rel_err(zg[clean], zo[clean])
    r["clean_frac"] = float(clean.mean())
    return r, new_o, info


def assert_clean(r, max_flip_frac=0.02, n=None):
    """All flips explained, all compared values within tolerance, and flips
    rare: at most max_flip_frac of the new particles (at least one, for tiny N)."""
    for key in ("anc_unexplained", "cand_unexplained", "sel_unexplained", "z_unexplained"):
        assert r.get(key, 0) == 0, r.line()
    for key in ("err_ell", "err_logw", "err_x", "err_z", "err_lam"):
        if key in r:
            assert r[key] <= TOL, r.line()
    floor = 1.0 / n if n else 0.0
    assert r["clean_frac"] >= 1.0 - max(max_flip_frac, floor), r.line()


def _inner_tie(model, st32, i, xt_i, u_in, b, j, M):
    """Whether inner point j of particle i lies within DELTA of the boundary
    of its chosen index b in the x-conditioned inner weights (FP64)."""
    kap = st32["lam"][i] + model.logpx(xt_i, st32["x"][i], st32["z"][i], st32["t"])
    wk, _, _ = weights_from_log(kap)
    C = np.cumsum(wk)
    Pj = ((j + u_in) * C[-1]) / M
    return abs(Pj - C[b]) <= DELTA * C[-1] or (b > 0 and abs(Pj - C[b - 1]) <= DELTA * C[-1])


def _inner_any_tie(model, st32, i, xt_i, u_in, M):
    kap = st32["lam"][i] + model.logpx(xt_i, st32["x"][i], st32["z"][i], st32["t"])
    wk, _, _ = weights_from_log(kap)
    C = np.cumsum(wk)
    Pj = ((np.arange(M) + u_in) * C[-1]) / M
    return bool(np.any(np.min(np.abs(Pj[:, None] - C[None, :]), axis=1) <= DELTA * C[-1]))


def compare_learned(model, st32, y32, seed, fid, mdn, g_state, g_logw, g_anc, g_comp, ess_frac):
    """Compare one learned step (the oracle takes the same network outputs
    mdn, FP32 values).  g_comp: the GPU's mixture component per
    pre-resampling particle."""
    from oracle import learned
    new_o, info = learned.step(model, st32, y32, seed, fid, mdn, ess_frac=ess_frac)
    N, M = st32["lam"].shape
    t = st32["t"] + 1
    r = Report()
    r["fallback"] = bool(info["fallback"])
    if info["fallback"]:
        return r, new_o, info
    u_mdn = P.uniform53(seed, fid, t, np.arange(N), P.MDN_U)
    u_in = P.uniform53(seed, fid, t, np.arange(N), P.INNER_U)
    logits = mdn[:, :4]
    bad_c = np.nonzero(g_comp != info["comp"])[0]
    r["comp_flips"] = len(bad_c)
    unexpl = 0
    for i in bad_c:
        wc, _, _ = weights_from_log(logits[i])
        unexpl += not near_tie(wc, u_mdn[i], 1, 0, info["comp"][i], g_comp[i])
    r["comp_unexplained"] = unexpl
    okc = g_comp == info["comp"]
    # outer log-weights: compared where the component agrees; a difference is
    # legitimate only where the particle's inner resampling has a near tie
    d = np.abs(g_logw - info["logw"]) / np.maximum(1.0, np.abs(info["logw"]))
    both_inf = np.isneginf(g_logw) & np.isneginf(info["logw"])
    d = np.where(both_inf, 0.0, d)
    badw = np.nonzero(okc & (d > TOL))[0]
    tie = [i for i in badw if _inner_any_tie(model, st32, i, info["xt"][i], u_in[i], M)]
    r["logw_off"] = len(badw)
    r["logw_unexplained"] = len(badw) - len(tie)
    mask = okc.copy()
    mask[tie] = False
    r["err_logw"] = float(np.max(d[mask])) if mask.any() else 0.0
    w_out, _, _ = weights_from_log(info["logw"])
    u_out = float(P.uniform53(seed, fid, t, 0, P.OUTER_U))
    A_o, A_g = info["A"], g_anc
    bad_anc = np.nonzero(A_o != A_g)[0]
    r["anc_flips"] = len(bad_anc)
    r["anc_unexplained"] = sum(not near_tie(w_out, u_out, N, k, A_o[k], A_g[k]) for k in bad_anc)
    good = (A_o == A_g) & okc[A_o]
    r["err_x"] = rel_err(g_state["x"][good], new_o["x"][good])
    zg, zo = g_state["z"], new_o["z"]
    dz = np.max(np.abs(zg - zo) / np.maximum(1.0, np.abs(zo)), axis=2)
    zflip = good[:, None] & (dz > TOL)
    r["z_flips"] = int(zflip.sum())
    unexpl = 0
    for k, j in zip(*np.nonzero(zflip)):
        i = A_o[k]
        unexpl += not _inner_tie(model, st32, i, info["xt"][i], u_in[i], info["binner"][i, j], j, M)
    r["z_unexplained"] = unexpl
    clean = good & ~zflip.any(axis=1)
    r["err_z"] = rel_err(zg[clean], zo[clean])
    r["err_lam"] = rel_err(g_state["lam"][clean], new_o["lam"][clean])
    r["clean_frac"] = float(clean.mean())
    return r, new_o, info


def assert_clean_learned(r, n=None, max_flip_frac=0.02):
    for key in ("comp_unexplained", "logw_unexplained", "anc_unexplained", "z_unexplained"):
        assert r.get(key, 0) == 0, r.line()
    for key in ("err_logw", "err_x", "err_z", "err_lam"):
        assert r[key] <= TOL, r.line()
    floor = 1.0 / n if n else 0.0
    assert r["clean_frac"] >= 1.0 - max(max_flip_frac, floor), r.line()


def compare_nested_weights(model, st32, y32, seed, fid, K, g_ell):
    """Compare the nested look-ahead weights of one step (K companions per
    candidate) with the oracle's.  A companion ancestor may flip where its
    systematic point lies within DELTA of a boundary of the candidate's
    conditioned cumulative weights; an ell mismatch must be explained by such
    a near tie.  Returns (report, oracle ell, rows with an explained flip)."""
    xla, ell_o, logw_o, comp, _ = ladpf.lookahead_nested(model, st32, y32, seed, fid, K)
    N, M = st32["lam"].shape
    t = st32["t"] + 1
    u = P.uniform53_ab(seed, fid, t, np.arange(N)[:, None], np.arange(M)[None, :], P.LA_B)
    r = Report()
    both_inf = np.isinf(g_ell) & np.isinf(ell_o) & (np.sign(g_ell) == np.sign(ell_o))
    d = np.where(both_inf, 0.0, np.abs(g_ell - ell_o) / np.maximum(1.0, np.abs(ell_o)))
    bad = np.argwhere(d > TOL)
    r["ell_off"] = len(bad)
    unexpl = 0
    tainted = np.zeros(N, dtype=bool)
    for i, m in bad:
        kap = st32["lam"][i] + model.logpx(xla[i, m], st32["x"][i], st32["z"][i], t - 1)
        wk, _, _ = weights_from_log(kap)
        C = np.cumsum(wk)
        Pk = ((np.arange(K) + u[i, m]) * C[-1]) / K
        near = np.min(np.abs(Pk[:, None] - C[None, :])) <= DELTA * C[-1]
        unexpl += not near
        tainted[i] = True
    r["ell_unexplained"] = int(unexpl)
    ok = ~both_inf & (d <= TOL)
    r["err_ell"] = float(np.max(d[ok])) if ok.any() else 0.0
    r["tainted_rows"] = int(tainted.sum())
    return r, ell_o, tainted
