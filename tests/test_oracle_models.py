"""Pins of the oracle's model densities and samplers (CPU only).

Each log density is compared with SciPy's library density of the same
distribution, and each sampler, fed zero noise, must return the transition
mean; fed unit noise it must move by the noise standard deviation.
"""
import math

import numpy as np
import pytest
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


def test_twodim_transition_is_the_joint_gaussian_of_table1():
    """Model 1 of Table 1.  The factorised transition p(x'|x,z) p(z'|x,x',z)
    of the oracle must be the joint law of Table 1: the pair of noises
    (x' - mean_x, z' - mean_z) is N(0, [[1, .1], [.1, 1]]).  Both densities
    are checked against SciPy's bivariate normal: log p(x'|.) from logpx, and
    the inner conditional from the sampler (affine in its normal), so a wrong
    conditional mean (a dropped v^x term, a wrong sign) or variance fails."""
    spec = S.twodim_table1()
    m = _model(spec)
    # (the library stores parameters in FP32; the spec rounds them once)
    cov = np.array([[1.0, 0.1], [0.1, 1.0]], dtype=np.float32).astype(np.float64)
    f12 = float(np.float32(1.2))
    g = np.random.default_rng(5)
    for _ in range(50):
        x, z, t = g.normal(size=1) * 3, g.normal(size=1) * 3, int(g.integers(0, 400))
        mean_x = x[0] + z[0] / (1 + z[0] ** 2)
        mean_z = x[0] + 0.5 * z[0] + 25 * z[0] / (1 + z[0] ** 2) + 8 * math.cos(f12 * t)
        vx, vz = g.normal(size=2) * 1.3
        xn = np.array([mean_x + vx])
        # z' = a + c * nu for the sampler: recover a and c, then the density
        a = m.fz(x, xn, z, np.zeros(1), t)[0]
        c = m.fz(x, xn, z, np.ones(1), t)[0] - a
        log_cond = stats.norm.logpdf(mean_z + vz, a, abs(c))
        joint = stats.multivariate_normal(mean=[0.0, 0.0], cov=cov).logpdf([vx, vz])
        assert np.isclose(float(m.logpx(xn, x, z)) + log_cond, joint, rtol=0, atol=1e-9)
    # the time-varying drift: 8 cos(1.2 t) with t the time the transition leaves
    x, z, xn = np.array([0.3]), np.array([-1.2]), np.array([0.1])
    d = m.fz(x, xn, z, np.zeros(1), 7)[0] - m.fz(x, xn, z, np.zeros(1), 2)[0]
    assert np.isclose(d, 8 * (math.cos(1.2 * 7) - math.cos(1.2 * 2)), atol=1e-5)


def test_twodim_likelihood_matches_scipy_and_integrates_to_one():
    spec = S.twodim_table1()
    m = _model(spec)
    g = np.random.default_rng(6)
    for _ in range(20):
        x, z, y = g.normal(size=1) * 4, g.normal(size=1) * 4, g.normal(size=1) * 3
        want = stats.norm.logpdf(y[0], math.atan(x[0]) + z[0] ** 2 / 20, 1.0)
        assert np.isclose(m.logpy(y, x, z), want)
    ys = np.linspace(-15, 25, 40001)[:, None]
    dens = np.exp(m.logpy(ys, np.array([0.7]), np.array([2.0])))
    assert abs(np.trapezoid(dens, ys[:, 0]) - 1.0) < 1e-6


def test_twodim_simulator_noise_covariance():
    """The simulator's own restatement of Table 1 (a separate module) draws
    noise pairs with the stated covariance."""
    spec = S.twodim_table1()
    xs, zs, _ = S.simulate(spec, 40000, 11)
    x, z = xs[:-1, 0], zs[:-1, 0]
    t = np.arange(len(x))
    vx = xs[1:, 0] - x - z / (1 + z * z)
    vz = zs[1:, 0] - (x + 0.5 * z + 25 * z / (1 + z * z) + 8 * np.cos(float(np.float32(1.2)) * t))
    c = np.cov(np.stack([vx, vz]))
    assert np.allclose(c, [[1.0, 0.1], [0.1, 1.0]], atol=0.03)


def test_twodim_time_convention_in_the_filters():
    """Table 1 writes z_{t+1} with 8 cos(1.2 t): the step that consumes y_t
    propagates out of time t - 1 (look-ahead draws and new clouds), the plain
    DPF's step t proposes t + 1 out of time t."""
    from oracle import dpf as odpf
    from oracle import ladpf
    from oracle import philox as P
    spec = S.twodim_table1()
    m = _model(spec)
    f12 = float(np.float32(1.2))
    st = ladpf.init_state(m, 3, 4, 9, 0)
    st["t"] = 4                                   # the step consumes y_5
    xla, zla, _, _ = ladpf.lookahead(m, st, np.array([0.2]), 9, 0)
    # the candidate's z normal follows its x normal in the one look-ahead draw
    nu_z = P.normals(9, 0, 5, np.arange(3)[:, None], np.arange(4)[None, :], P.LA_X, 2)[..., 1:]
    x, z = st["x"][:, None, :], st["z"]
    vx = xla - x - z / (1 + z * z)
    want = x + 0.5 * z + 25 * z / (1 + z * z) + 8 * math.cos(f12 * 4) + 0.1 * vx + math.sqrt(0.99) * nu_z
    assert np.allclose(zla, want, atol=1e-6)
    # plain: step t = 5 proposes z_6 out of time 5
    xs, zs = st["x"], st["z"]
    xn, zn, anc, b, _ = odpf.propose(m, xs, zs, np.full((3, 4), -math.log(4)), np.arange(3), 5, 9, 0)
    nu = np.stack([P.normals(9, 0, 5, k, np.arange(4), P.DPF_Z, 1) for k in range(3)])
    zp = np.stack([zs[k, b[k]] for k in range(3)])
    vx = xn[:, None, :] - xs[:, None, :] - zp / (1 + zp * zp)
    want = xs[:, None, :] + 0.5 * zp + 25 * zp / (1 + zp * zp) + 8 * math.cos(f12 * 5) + 0.1 * vx \
        + math.sqrt(0.99) * nu
    assert np.allclose(zn, want, atol=1e-6)


def test_fourdim_transition_and_likelihood_match_table1_laws():
    """Model 2 of Table 1.  log p(x'|x) against SciPy with the sin t drift;
    the inner sampler is affine in its normals, z' = a + C nu: the noise pair
    (w1, w2) it implies (w2 taken from z2' minus z1' and the drift, as Table
    1 writes z2' in terms of the new z1') must have covariance
    [[1, 0.1], [0.1, 10]] and zero mean; the likelihood against SciPy."""
    spec = S.fourdim_table1()
    m = _model(spec)
    f12 = float(np.float32(1.2))
    g = np.random.default_rng(8)
    for _ in range(30):
        x, z, t = g.normal(size=2) * 3, g.normal(size=2) * 3, int(g.integers(0, 400))
        xn = g.normal(size=2) * 4
        want = (stats.norm.logpdf(xn[0], 0.5 * x[0] + 8 * math.sin(t), 1.0)
                + stats.norm.logpdf(xn[1], 0.4 * x[0] + 0.5 * x[1], 1.0))
        assert np.isclose(m.logpx(xn, x, z, t), want)
        base = m.fz(x, xn, z, np.zeros(2), t)

        def noise(zn):
            w1 = zn[0] - (z[0] + z[1] / (1 + z[1] ** 2))
            w2 = zn[1] - (zn[0] + 0.5 * z[1] + 25 * z[1] / (1 + z[1] ** 2) + 8 * math.cos(f12 * t))
            return np.array([w1, w2])
        assert np.allclose(noise(base), 0.0, atol=1e-9)
        C = np.stack([noise(m.fz(x, xn, z, np.eye(2)[k], t)) for k in range(2)], axis=1)
        cov = np.array([[1.0, 0.1], [0.1, 10.0]], dtype=np.float32).astype(np.float64)
        assert np.allclose(C @ C.T, cov, atol=1e-9)
        y = g.normal(size=1) * 3
        h = (x[0] + x[1]) / (1 + x[0] ** 2) + math.atan(z[0]) + z[1] ** 2 / 20
        assert np.isclose(m.logpy(y, x, z), stats.norm.logpdf(y[0], h, 1.0))


def test_fourdim_simulator_noise_covariance():
    spec = S.fourdim_table1()
    xs, zs, _ = S.simulate(spec, 40000, 12)
    t = np.arange(len(xs) - 1)
    x, z = xs[:-1], zs[:-1]
    v1 = xs[1:, 0] - 0.5 * x[:, 0] - 8 * np.sin(t)
    v2 = xs[1:, 1] - 0.4 * x[:, 0] - 0.5 * x[:, 1]
    w1 = zs[1:, 0] - z[:, 0] - z[:, 1] / (1 + z[:, 1] ** 2)
    w2 = zs[1:, 1] - zs[1:, 0] - 0.5 * z[:, 1] - 25 * z[:, 1] / (1 + z[:, 1] ** 2) \
        - 8 * np.cos(float(np.float32(1.2)) * t)
    c = np.cov(np.stack([v1, v2, w1, w2]))
    want = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0.1], [0, 0, 0.1, 10]])
    assert np.all(np.abs(c - want) <= 0.05 * np.sqrt(np.outer(np.diag(want), np.diag(want))))


@pytest.mark.parametrize("zfirst,after,q", [(False, True, (1.0, 1.0, 0.1)), (True, False, (1.0, 1.0, 0.1)),
                                             (True, True, (1.0, 1.0, 0.1)), (False, False, (1.3, 0.7, 0.2)),
                                             (True, False, (1.3, 0.7, 0.2)), (True, True, (1.3, 0.7, 0.2))])
def test_twodim_orders_and_change_point_are_the_joint_gaussian(zfirst, after, q):
    """Both sampling orders of model 1 factorise the same joint transition:
    log p(o'|o, i) + log p(i'|o, i, o') must equal SciPy's bivariate normal
    of the noise pair (v^x, v^z) ~ N(0, [[1, .1], [.1, 1]]) around the means
    of Table 1 (and around the same means with other noise covariances) --
    before the change point x' = x + z/(1+z^2) and
    z' = x + .5 z + 25 z/(1+z^2) + 8 cos(1.2 t); from tswap on the two laws
    swapped (x' = z + .5 x + 25 x/(1+x^2) + 8 cos(1.2 t), z' = z + x/(1+x^2)).
    With z first the outer state is z and the inner one x."""
    tswap = 300
    spec = S.twodim_table1(qx=q[0], qz=q[1], cxz=q[2], tswap=tswap, zfirst=zfirst)
    m = _model(spec)
    cov = np.array([[q[0], q[2]], [q[2], q[1]]], dtype=np.float32).astype(np.float64)
    f12 = float(np.float32(1.2))
    g = np.random.default_rng(7 + 2 * zfirst + after)
    for _ in range(50):
        x, z = g.normal() * 3, g.normal() * 3
        t = int(g.integers(tswap, tswap + 200)) if after else int(g.integers(0, tswap))
        if after:
            mean_x = z + 0.5 * x + 25 * x / (1 + x * x) + 8 * math.cos(f12 * t)
            mean_z = z + x / (1 + x * x)
        else:
            mean_x = x + z / (1 + z * z)
            mean_z = x + 0.5 * z + 25 * z / (1 + z * z) + 8 * math.cos(f12 * t)
        vx, vz = g.normal(size=2) * 1.3
        xn, zn = mean_x + vx, mean_z + vz
        o, i, on, inn = (z, x, zn, xn) if zfirst else (x, z, xn, zn)
        o, i, on = np.array([o]), np.array([i]), np.array([on])
        a = m.fz(o, on, i, np.zeros(1), t)[0]
        c = m.fz(o, on, i, np.ones(1), t)[0] - a
        log_cond = stats.norm.logpdf(inn, a, abs(c))
        joint = stats.multivariate_normal(mean=[0.0, 0.0], cov=cov).logpdf([vx, vz])
        assert np.isclose(float(m.logpx(on, o, i, t)) + log_cond, joint, rtol=0, atol=1e-9)
        # the outer sampler is its density's mean plus its scale times the normal
        assert np.isclose(m.fx(o, i, np.zeros(1), t)[0], mean_z if zfirst else mean_x, atol=1e-12)
    # the observation, whichever block is outer
    yv = np.array([0.4])
    o, i = (np.array([1.5]), np.array([-0.7])) if zfirst else (np.array([-0.7]), np.array([1.5]))
    assert np.isclose(m.logpy(yv, o, i), stats.norm.logpdf(0.4, math.atan(-0.7) + 1.5 ** 2 / 20, 1.0))


def test_twodim_simulator_swaps_the_laws_at_the_change_point():
    spec = S.twodim_table1(tswap=500)
    xs, zs, _ = S.simulate(spec, 20000, 12)
    f12 = float(np.float32(1.2))
    x, z = xs[:-1, 0], zs[:-1, 0]
    t = np.arange(len(x))
    a = t >= 500
    vx = np.where(a, xs[1:, 0] - (z + 0.5 * x + 25 * x / (1 + x * x) + 8 * np.cos(f12 * t)),
                  xs[1:, 0] - x - z / (1 + z * z))
    vz = np.where(a, zs[1:, 0] - z - x / (1 + x * x),
                  zs[1:, 0] - (x + 0.5 * z + 25 * z / (1 + z * z) + 8 * np.cos(f12 * t)))
    c = np.cov(np.stack([vx[a], vz[a]]))
    assert np.allclose(c, [[1.0, 0.1], [0.1, 1.0]], atol=0.04)
    assert np.max(np.abs(vx[~a])) < 6 and np.max(np.abs(vz[~a])) < 6
    # the z-first spec simulates the same truth and observations
    xs2, zs2, ys2 = S.simulate(S.twodim_table1(tswap=500, zfirst=True), 300, 12)
    _, _, ys = S.simulate(spec, 300, 12)
    assert np.array_equal(ys, ys2) and np.array_equal(xs[:301], xs2) and np.array_equal(zs[:301], zs2)
