"""Closed-form filters used to pin the particle oracle (FP64).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

For the linear-Gaussian instance of Eq. (1) the posterior p(x_t, z_t | y_{1:t})
is Gaussian and the Kalman filter computes it exactly; the filtered means,
variances and the log evidence log p(y_{1:T}) are the targets the particle
filters must approach as N and M grow.

Joint state s = [x; z].  Substituting x_{t+1} into the z transition:
    s' = F s + G v,   F = [[Ax, Cxz], [Bzx Ax, Az + Bzx Cxz]],
    G = [[I, 0], [Bzx, I]],  v ~ N(0, diag(qx I, qz I)),
    y  = H s + e,     H = [Hx, Hz],  e ~ N(0, r I),  s_0 ~ N(0, I).

The conditional filter of z given an x path (the exact inner filter of a
Rao-Blackwellised particle filter, Section 1) is ``conditional_kf_step``.
"""
import numpy as np


def joint_matrices(m):
    dx, dz = m.dx, m.dz
    F = np.block([[m.Ax, m.Cxz], [m.Bzx @ m.Ax, m.Az + m.Bzx @ m.Cxz]])
    G = np.block([[np.eye(dx), np.zeros((dx, dz))], [m.Bzx, np.eye(dz)]])
    Qv = np.diag(np.r_[np.full(dx, m.qx), np.full(dz, m.qz)])
    Q = G @ Qv @ G.T
    H = np.hstack([m.Hx, m.Hz])
    R = m.r * np.eye(m.dy)
    return F, Q, H, R


def kalman_filter(m, ys):
    """Filtered means (T, dx+dz), covariances (T, d, d), and log p(y_{1:T})."""
    F, Q, H, R = joint_matrices(m)
    d = F.shape[0]
    mu = np.zeros(d)
    P = np.eye(d)
    means, covs, ll = [], [], 0.0
    for y in ys:
        mu = F @ mu
        P = F @ P @ F.T + Q
        S = H @ P @ H.T + R
        innov = np.asarray(y) - H @ mu
        Sinv = np.linalg.inv(S)
        K = P @ H.T @ Sinv
        sign, logdet = np.linalg.slogdet(2.0 * np.pi * S)
        ll += -0.5 * (logdet + innov @ Sinv @ innov)
        mu = mu + K @ innov
        P = (np.eye(d) - K @ H) @ P
        P = 0.5 * (P + P.T)
        means.append(mu.copy())
        covs.append(P.copy())
    return np.asarray(means), np.asarray(covs), ll


def conditional_kf_step(m, mu, P, x_prev, x_new, y):
    """One step of the exact filter of z given the x path and y (linear-Gaussian).

    (a) x_t = Ax x_{t-1} + Cxz z_{t-1} + v observes z_{t-1}: condition
        N(mu, P) on it (the extra factor of eq:qnobar); identity if Cxz = 0.
    (b) predict z_t = Az z_{t-1} + Bzx x_t + w.
    (c) update with y_t = Hx x_t + Hz z_t + e.
    Returns (mu_t, P_t).
    """
    dz = m.dz
    S1 = m.Cxz @ P @ m.Cxz.T + m.qx * np.eye(m.dx)
    K1 = P @ m.Cxz.T @ np.linalg.inv(S1)
    mu = mu + K1 @ (x_new - m.Ax @ x_prev - m.Cxz @ mu)
    P = P - K1 @ m.Cxz @ P
    mu_p = m.Az @ mu + m.Bzx @ x_new
    P_p = m.Az @ P @ m.Az.T + m.qz * np.eye(dz)
    S = m.Hz @ P_p @ m.Hz.T + m.r * np.eye(m.dy)
    K = P_p @ m.Hz.T @ np.linalg.inv(S)
    mu_t = mu_p + K @ (y - m.Hx @ x_new - m.Hz @ mu_p)
    P_t = (np.eye(dz) - K @ m.Hz) @ P_p
    return mu_t, 0.5 * (P_t + P_t.T)
