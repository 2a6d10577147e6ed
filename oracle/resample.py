"""Resampling and log-weight helpers, oracle side (FP64).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Section 2 calls steps 2 and 6 of the DPF (Fig. 2) and step 3 of the
look-ahead DPF (Fig. 4) "standard resampling steps" without fixing a scheme.
Both sides use systematic resampling, written out here from its definition:

    C_i = w_0 + ... + w_i            (serial cumulative sum, FP64)
    P_k = ((k + u) * C_{n-1}) / n_out    for k = 0 .. n_out-1
    A_k = min { i : C_i > P_k }      (first index strictly above the point)

evaluated left to right in IEEE double precision.  If rounding pushes a
point to or past the total, the index is the first i with C_i >= C_{n-1};
the strict rule never selects a zero weight.  A single inverse-CDF draw is
the same rule with n_out = 1.

Log-weights are turned into weights as w_i = exp(lw_i - max finite lw).  A
non-finite log-weight (NaN or +-inf) counts as weight zero and raises the
NONFINITE flag (NaN and +inf only); if no log-weight is finite the weights
fall back to uniform and DEGENERATE is raised.
"""
import math

import numpy as np

FLAG_DEGENERATE_OUTER = 1
FLAG_DEGENERATE_INNER = 2
FLAG_NONFINITE = 4
FLAG_FALLBACK = 8


def weights_from_log(lw):
    """Return (w, degenerate, nonfinite) for a vector of log-weights."""
    lw = np.asarray(lw, dtype=np.float64)
    finite = np.isfinite(lw)
    nonfinite = bool(np.any(np.isnan(lw) | (lw == np.inf)))
    if not finite.any():
        return np.ones_like(lw), True, nonfinite
    m = np.max(lw[finite])
    w = np.zeros_like(lw)
    w[finite] = np.exp(lw[finite] - m)
    return w, False, nonfinite


def logsumexp(a):
    """log sum exp over the last axis, ignoring non-finite entries.

    Returns -inf for a row with no finite entry.
    """
    a = np.asarray(a, dtype=np.float64)
    finite = np.isfinite(a)
    safe = np.where(finite, a, -np.inf)
    m = np.max(safe, axis=-1, keepdims=True)
    m_ok = np.where(np.isfinite(m), m, 0.0)
    s = np.sum(np.where(finite, np.exp(safe - m_ok), 0.0), axis=-1)
    with np.errstate(divide="ignore"):
        out = m_ok[..., 0] + np.log(s)
    return np.where(np.any(finite, axis=-1), out, -np.inf)


def systematic(w, n_out, u):
    """Systematic resampling indices (int64, non-decreasing) for weights w."""
    w = np.asarray(w, dtype=np.float64)
    C = np.cumsum(w)  # sequential accumulation, left to right
    total = C[-1]
    k = np.arange(n_out, dtype=np.float64)
    P = ((k + u) * total) / float(n_out)
    A = np.searchsorted(C, P, side="right")
    last = np.searchsorted(C, total, side="left")
    return np.minimum(A, last).astype(np.int64)


def systematic_log(lw, n_out, u):
    """Systematic resampling from log-weights; returns (A, degenerate, nonfinite)."""
    w, deg, nonf = weights_from_log(lw)
    return systematic(w, n_out, u), deg, nonf


def offspring_counts(A, n):
    return np.bincount(np.asarray(A, dtype=np.int64), minlength=n)


def normalise_log(a):
    """a - logsumexp(a) per row; a row with no finite entry becomes uniform.

    Returns (normalised, degenerate_rows_mask).
    """
    a = np.asarray(a, dtype=np.float64)
    lse = logsumexp(a)
    deg = ~np.isfinite(lse)
    n = a.shape[-1]
    out = np.where(np.isfinite(a), a - np.where(deg, 0.0, lse)[..., None], -np.inf)
    out = np.where(deg[..., None], -math.log(n), out)
    return out, deg
