"""Pins of the oracle's model densities and samplers (CPU only).

Each log density is compared with SciPy's library density of the same
distribution, and each sampler, fed zero noise, must return the transition
mean; fed unit noise it must move by the noise standard deviation.
"""
import math

import numpy as np
from scipy import stats

import dpf_synth as S
from oracle.models import make_model


def _model(spec):
    return make_model(spec.kind, spec.dx, spec.dz, spec.dy, spec.blob)


def test_lingauss_densities_match_scipy():
    for coupled in (False, True):
        spec = S.lingauss_c1(coupled)
        m = _model(spec)
        g = np.random.default_rng(0)
        for _ in range(20):
            x, z = g.normal(size=1), g.normal(size=2)
            xn, y = g.normal(size=1), g.normal(size=1)
            mean_x = 0.9 * x[0] + (0.2 * z[0] if coupled else 0.0)
            assert np.isclose(m.logpx(xn, x, z), stats.norm.logpdf(xn[0], mean_x, math.sqrt(0.1)))
            mean_y = x[0] + z[0] + 0.5 * z[1]
            assert np.isclose(m.logpy(y, x, z), stats.norm.logpdf(y[0], mean_y, math.sqrt(0.2)))
            zn = m.fz(x, xn, z, np.zeros(2))
            assert np.allclose(zn, [0.8 * z[0] + 0.1 * z[1] + 0.5 * xn[0], 0.7 * z[1] + 0.5 * xn[0]])
            zn1 = m.fz(x, xn, z, np.array([1.0, -1.0]))
            assert np.allclose(zn1 - zn, [math.sqrt(0.1), -math.sqrt(0.1)])


def test_nonlin_densities_match_scipy():
    spec = S.nonlin_c2(3)
    m = _model(spec)
    W = spec.blob[3:3 + 16].reshape(8, 2)
    g = np.random.default_rng(1)
    for _ in range(10):
        x, z = g.normal(size=2) * 3, g.normal(size=8)
        xn, y = g.normal(size=2) * 3, g.normal(size=8)
        mx = 0.5 * x + 25 * x / (1 + x * x)
        assert np.isclose(m.logpx(xn, x, z), stats.multivariate_normal.logpdf(xn, mx, np.eye(2)))
        my = z + 0.05 * np.array([x[k % 2] ** 2 for k in range(8)])
        assert np.isclose(m.logpy(y, x, z), stats.multivariate_normal.logpdf(y, my, 0.5 * np.eye(8)))
        zn = m.fz(x, xn, z, np.zeros(8))
        assert np.allclose(zn, np.tanh(W @ xn) + 0.9 * z)
        assert np.allclose(m.fx(x, z, np.ones(2)) - mx, 1.0)
    spec1 = S.nonlin_c2(3, bmode=1)
    m1 = _model(spec1)
    x, z, y = g.normal(size=2), g.normal(size=8), g.normal(size=8)
    my = z + 0.05 * np.dot(x, x)
    assert np.isclose(m1.logpy(y, x, z), stats.multivariate_normal.logpdf(y, my, 0.5 * np.eye(8)))


def test_highdim_mixture_likelihood_matches_scipy():
    spec = S.highdim_c4(2, dx=4, dz=16, dy=8)
    m = _model(spec)
    g = np.random.default_rng(2)
    C = m.C
    for _ in range(5):
        x, z, y = g.normal(size=4), g.normal(size=16), g.normal(size=8) * 2
        e = y - C @ z
        sd = math.sqrt(0.3)
        dens = 0.99 * stats.norm.pdf(e, 0, sd) + 0.01 * stats.t.pdf(e / sd, 3) / sd
        assert np.isclose(m.logpy(y, x, z), np.sum(np.log(dens)), rtol=1e-12)
        # t_3 density in closed form: (2 / (pi sqrt 3)) (1 + s^2/3)^-2
        s = 0.7
        assert np.isclose(stats.t.pdf(s, 3), 2 / (math.pi * math.sqrt(3)) * (1 + s * s / 3) ** -2)
    # tridiagonal A, spectral radius 0.95 (up to the FP32 rounding of the entries)
    assert np.allclose(np.triu(m.A, 2), 0) and np.allclose(np.tril(m.A, -2), 0)
    assert abs(np.max(np.abs(np.linalg.eigvals(m.A))) - 0.95) < 1e-5
    zn = m.fz(None, np.array([0.1, 0.2, 0.3, 0.4]), np.ones(16), np.zeros(16))
    assert np.allclose(zn, m.A @ np.ones(16) + m.B @ np.sin([0.1, 0.2, 0.3, 0.4]))
    specg = S.highdim_c4(2, dx=4, dz=16, dy=8, gaussian_only=True)
    mg = _model(specg)
    assert np.isclose(mg.logpy(y, x, z), stats.multivariate_normal.logpdf(y, C @ z, 0.3 * np.eye(8)))


def test_broadcasting_shapes():
    spec = S.nonlin_c2(1)
    m = _model(spec)
    x = np.zeros((5, 1, 2))
    z = np.zeros((5, 7, 8))
    nu = np.zeros((5, 7, 2))
    assert m.fx(x, z, nu).shape == (5, 7, 2)
    assert m.logpy(np.zeros(8), m.fx(x, z, nu), z).shape == (5, 7)
