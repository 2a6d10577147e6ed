"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

This module only *generates inputs*: model parameter blobs (drawn with a
NumPy PCG64 stream from ``param_seed``), simulated trajectories and
observations (PCG64 from ``data_seed``), ragged batch shapes and random
weight arrays.  It contains none of the filter's arithmetic; the
simulator below is its own short restatement of each model's generative
equations (Eq. (1) of the paper), used only to produce truth and
observations.

Parameter blob layouts are those of the library interface (include/dpf.h):

LINGAUSS: Ax[dx*dx] Cxz[dx*dz] qx Az[dz*dz] Bzx[dz*dx] qz Hx[dy*dx] Hz[dy*dz] r
NONLIN:   a b qx W[dz*dx] rho qz c r bmode
HIGHDIM:  a b qx Alo[dz-1] Adiag[dz] Aup[dz-1] B[dz*dx] qz C[dy*dz] r eps nu gonly
TWODIM:   qx qz cxz rho b amp freq r tswap   (TWODIM_ZFIRST: the same blob)
FOURDIM:  a1 bs c21 a2 qx1 qx2 qz1 qz2 cz rho b amp freq r
"""
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

LINGAUSS, NONLIN, HIGHDIM, TWODIM, FOURDIM, TWODIM_ZFIRST = 1, 2, 3, 4, 5, 6


@dataclass
class ModelSpec:
    kind: int
    dx: int
    dz: int
    dy: int
    blob: np.ndarray

    @property
    def name(self):
        return {LINGAUSS: "lingauss", NONLIN: "nonlin", HIGHDIM: "highdim", TWODIM: "twodim",
                FOURDIM: "fourdim", TWODIM_ZFIRST: "twodim_zfirst"}[self.kind]


def lingauss_c1(coupled: bool = False) -> ModelSpec:
    """dx=1, dz=2, dy=1 linear-Gaussian workload.

    x_t = 0.9 x_{t-1} (+ 0.2 z_{1,t-1} when coupled) + N(0, 0.1)
    z_t = [[0.8, 0.1], [0, 0.7]] z_{t-1} + 0.5 x_t [1, 1] + N(0, 0.1 I)
    y_t = [1, 0.5] z_t + x_t + N(0, 0.2)
    """
    Ax = [0.9]
    Cxz = [0.2, 0.0] if coupled else [0.0, 0.0]
    Az = [0.8, 0.1, 0.0, 0.7]
    Bzx = [0.5, 0.5]
    Hx = [1.0]
    Hz = [1.0, 0.5]
    blob = np.array(Ax + Cxz + [0.1] + Az + Bzx + [0.1] + Hx + Hz + [0.2], dtype=np.float64)
    return ModelSpec(LINGAUSS, 1, 2, 1, blob)


def twodim_table1(qx: float = 1.0, qz: float = 1.0, cxz: float = 0.1, tswap: float = np.inf,
                  zfirst: bool = False) -> ModelSpec:
    """Model 1 of Table 1 (the 2-dimensional example), dx = dz = dy = 1:

    x_{t+1} = x_t + z_t / (1 + z_t^2) + v^x_t
    z_{t+1} = x_t + 0.5 z_t + 25 z_t / (1 + z_t^2) + 8 cos(1.2 t) + v^z_t
    y_t = atan(x_t) + z_t^2 / 20 + e_t
    (v^x, v^z) ~ N(0, [[qx, cxz], [cxz, qz]]) (Table 1: 1, 1, 0.1), e ~ N(0, 1).
    From t >= tswap on the two transition laws are swapped (x' = z + 0.5 x +
    25 x / (1 + x^2) + 8 cos(1.2 t) + v^x, z' = z + x / (1 + x^2) + v^z).
    zfirst: the decomposition that samples z first (outer z, inner x); the
    simulated truth and observations are the same.  Parameters are rounded
    to FP32 once, as the library stores them.
    """
    blob = np.array([qx, qz, cxz, 0.5, 25.0, 8.0, 1.2, 1.0, tswap], dtype=np.float32).astype(np.float64)
    return ModelSpec(TWODIM_ZFIRST if zfirst else TWODIM, 1, 1, 1, blob)


def fourdim_table1() -> ModelSpec:
    """Model 2 of Table 1 (the 4-dimensional example), dx = dz = 2, dy = 1:

    x1' = 0.5 x1 + 8 sin t + v1,  x2' = 0.4 x1 + 0.5 x2 + v2
    z1' = z1 + z2 / (1 + z2^2) + w1
    z2' = z1' + 0.5 z2 + 25 z2 / (1 + z2^2) + 8 cos(1.2 t) + w2
    y = (x1 + x2) / (1 + x1^2) + atan(z1) + z2^2 / 20 + e
    v ~ N(0, I), (w1, w2) ~ N(0, [[1, 0.1], [0.1, 10]]), e ~ N(0, 1).
    """
    blob = np.array([0.5, 8.0, 0.4, 0.5, 1.0, 1.0, 1.0, 10.0, 0.1, 0.5, 25.0, 8.0, 1.2, 1.0],
                    dtype=np.float32).astype(np.float64)
    return ModelSpec(FOURDIM, 2, 2, 1, blob)


def nonlin_c2(param_seed: int = 1, dx: int = 2, dz: int = 8, bmode: int = 0) -> ModelSpec:
    """Nonlinear workload: growth-model x, tanh-coupled z, z plus 0.05 x^2 observed.

    W has entries ~ N(0, 1/dx), drawn from ``param_seed``.
    """
    rng = np.random.Generator(np.random.PCG64(param_seed))
    W = rng.normal(0.0, np.sqrt(1.0 / dx), size=(dz, dx)).astype(np.float32).astype(np.float64)
    blob = np.concatenate([[0.5, 25.0, 1.0], W.ravel(), [0.9, 0.05, 0.05, 0.5, float(bmode)]])
    return ModelSpec(NONLIN, dx, dz, dz, blob.astype(np.float64))


def highdim_c4(param_seed: int = 1, dx: int = 4, dz: int = 64, dy: int = 32,
               gaussian_only: bool = False) -> ModelSpec:
    """High-dimensional inner block: tridiagonal A (spectral radius 0.95),
    B ~ N(0, 0.1), C ~ N(0, 1/dz), Student-t(3) outlier mixture likelihood."""
    rng = np.random.Generator(np.random.PCG64(param_seed))
    lo = rng.normal(size=dz - 1)
    dg = rng.normal(size=dz)
    up = rng.normal(size=dz - 1)
    A = np.diag(dg) + np.diag(lo, -1) + np.diag(up, 1)
    rho = np.max(np.abs(np.linalg.eigvals(A)))
    s = 0.95 / rho
    lo, dg, up = lo * s, dg * s, up * s
    # The library stores parameters in FP32; round them once so that both
    # sides see the same values.
    lo, dg, up = (v.astype(np.float32).astype(np.float64) for v in (lo, dg, up))
    B = rng.normal(0.0, np.sqrt(0.1), size=(dz, dx)).astype(np.float32).astype(np.float64)
    C = rng.normal(0.0, np.sqrt(1.0 / dz), size=(dy, dz)).astype(np.float32).astype(np.float64)
    blob = np.concatenate([[0.5, 25.0, 1.0], lo, dg, up, B.ravel(), [0.02], C.ravel(),
                           [0.3, 0.01, 3.0, 1.0 if gaussian_only else 0.0]])
    return ModelSpec(HIGHDIM, dx, dz, dy, blob.astype(np.float64))


# ---------------------------------------------------------------- simulator
def _sim_fns(spec: ModelSpec):
    """fx(x, z, g), fz(x, xn, z, g, t), hy(x, z, g); t is the time of the
    state the transition leaves."""
    dx, dz, dy, b = spec.dx, spec.dz, spec.dy, spec.blob
    if spec.kind == LINGAUSS:
        o = 0
        Ax = b[o:o + dx * dx].reshape(dx, dx); o += dx * dx
        Cxz = b[o:o + dx * dz].reshape(dx, dz); o += dx * dz
        qx = b[o]; o += 1
        Az = b[o:o + dz * dz].reshape(dz, dz); o += dz * dz
        Bzx = b[o:o + dz * dx].reshape(dz, dx); o += dz * dx
        qz = b[o]; o += 1
        Hx = b[o:o + dy * dx].reshape(dy, dx); o += dy * dx
        Hz = b[o:o + dy * dz].reshape(dy, dz); o += dy * dz
        r = b[o]
        fx = lambda x, z, g, t: Ax @ x + Cxz @ z + np.sqrt(qx) * g.normal(size=dx)
        fz = lambda x, xn, z, g, t: Az @ z + Bzx @ xn + np.sqrt(qz) * g.normal(size=dz)
        hy = lambda x, z, g: Hx @ x + Hz @ z + np.sqrt(r) * g.normal(size=dy)
        return fx, fz, hy
    if spec.kind == NONLIN:
        a, bb, qx = b[0], b[1], b[2]
        W = b[3:3 + dz * dx].reshape(dz, dx)
        rho, qz, c, r, bmode = b[3 + dz * dx:3 + dz * dx + 5]
        fx = lambda x, z, g, t: a * x + bb * x / (1 + x * x) + np.sqrt(qx) * g.normal(size=dx)
        fz = lambda x, xn, z, g, t: np.tanh(W @ xn) + rho * z + np.sqrt(qz) * g.normal(size=dz)

        def hy(x, z, g):
            off = c * x[np.arange(dy) % dx] ** 2 if bmode == 0 else c * np.dot(x, x)
            return z + off + np.sqrt(r) * g.normal(size=dy)
        return fx, fz, hy
    if spec.kind == HIGHDIM:
        a, bb, qx = b[0], b[1], b[2]
        o = 3
        lo = b[o:o + dz - 1]; o += dz - 1
        dg = b[o:o + dz]; o += dz
        up = b[o:o + dz - 1]; o += dz - 1
        A = np.diag(dg) + np.diag(lo, -1) + np.diag(up, 1)
        B = b[o:o + dz * dx].reshape(dz, dx); o += dz * dx
        qz = b[o]; o += 1
        C = b[o:o + dy * dz].reshape(dy, dz); o += dy * dz
        r, eps, nu, gonly = b[o:o + 4]
        fx = lambda x, z, g, t: a * x + bb * x / (1 + x * x) + np.sqrt(qx) * g.normal(size=dx)
        fz = lambda x, xn, z, g, t: A @ z + B @ np.sin(xn) + np.sqrt(qz) * g.normal(size=dz)

        def hy(x, z, g):
            e = np.sqrt(r) * g.normal(size=dy)
            if not gonly:
                out = g.random(size=dy) < eps
                e = np.where(out, np.sqrt(r) * g.standard_t(nu, size=dy), e)
            return C @ z + e
        return fx, fz, hy
    if spec.kind in (TWODIM, TWODIM_ZFIRST):
        qx, qz, cxz, rho, bb, amp, freq, r, tswap = b
        slow = lambda s_, o_: s_ + o_ / (1 + o_ * o_)
        grow = lambda g_, o_, t: o_ + rho * g_ + bb * g_ / (1 + g_ * g_) + amp * np.cos(freq * t)
        mx = lambda x, z, t: grow(x, z, t) if t >= tswap else slow(x, z)
        mz = lambda x, z, t: slow(z, x) if t >= tswap else grow(z, x, t)
        # the noise pair drawn jointly: v^x first, then v^z given v^x
        fx = lambda x, z, g, t: mx(x, z, t) + np.sqrt(qx) * g.normal(size=1)

        def fz(x, xn, z, g, t):
            vx = xn - mx(x, z, t)
            vz = cxz / qx * vx + np.sqrt(qz - cxz * cxz / qx) * g.normal(size=1)
            return mz(x, z, t) + vz
        hy = lambda x, z, g: np.arctan(x) + z * z / 20 + np.sqrt(r) * g.normal(size=1)
        return fx, fz, hy
    if spec.kind == FOURDIM:
        a1, bs, c21, a2, qx1, qx2, qz1, qz2, cz, rho, bb, amp, freq, r = b

        def fx(x, z, g, t):
            v = g.normal(size=2) * np.sqrt([qx1, qx2])
            return np.array([a1 * x[0] + bs * np.sin(t), c21 * x[0] + a2 * x[1]]) + v

        def fz(x, xn, z, g, t):
            w = g.multivariate_normal([0.0, 0.0], [[qz1, cz], [cz, qz2]])
            z1 = z[0] + z[1] / (1 + z[1] ** 2) + w[0]
            return np.array([z1, z1 + rho * z[1] + bb * z[1] / (1 + z[1] ** 2) + amp * np.cos(freq * t) + w[1]])
        hy = lambda x, z, g: (np.array([(x[0] + x[1]) / (1 + x[0] ** 2) + np.arctan(z[0]) + z[1] ** 2 / 20])
                              + np.sqrt(r) * g.normal(size=1))
        return fx, fz, hy
    raise ValueError(spec.kind)


def simulate(spec: ModelSpec, T: int, data_seed: int):
    """Truth x_0..x_T, z_0..z_T and observations y_1..y_T (PCG64 stream)."""
    g = np.random.Generator(np.random.PCG64(data_seed))
    fx, fz, hy = _sim_fns(spec)
    x = g.normal(size=spec.dx)
    z = g.normal(size=spec.dz)
    xs, zs, ys = [x], [z], []
    for s in range(T):
        xn = fx(x, z, g, s)
        zn = fz(x, xn, z, g, s)
        ys.append(hy(xn, zn, g))
        x, z = xn, zn
        xs.append(x)
        zs.append(z)
    return np.asarray(xs), np.asarray(zs), np.asarray(ys)


# ------------------------------------------------------------ ragged batches
@dataclass
class RaggedBatch:
    N: np.ndarray
    M: np.ndarray
    T: np.ndarray
    data_seeds: np.ndarray


def ragged_batch(F: int = 1024, seed: int = 7, n_range=(256, 4096), m_choices=(32, 64, 128),
                 t_range=(50, 500), data_seed_base: int = 100000) -> RaggedBatch:
    """Per-filter sizes: N log-uniform in n_range (rounded), M uniform over
    m_choices, T uniform integer in t_range (inclusive)."""
    g = np.random.Generator(np.random.PCG64(seed))
    lo, hi = np.log(n_range[0]), np.log(n_range[1])
    N = np.rint(np.exp(g.uniform(lo, hi, size=F))).astype(np.int32)
    M = np.asarray(m_choices, dtype=np.int32)[g.integers(0, len(m_choices), size=F)]
    T = g.integers(t_range[0], t_range[1] + 1, size=F).astype(np.int32)
    return RaggedBatch(N, M, T, data_seed_base + np.arange(F, dtype=np.int64))


# ------------------------------------------------------ resampling corpora
def weight_corpus(seed: int, n: int, kind: str) -> np.ndarray:
    """Non-negative float64 weight arrays of assorted shapes for resampling tests.

    kinds: 'lognormal', 'equal', 'dominant', 'zeros' (about half exactly 0),
    'tiny' (spread over 600 decades of magnitude, many underflow to 0 in FP32
    but not in FP64), 'single' (one non-zero).
    """
    g = np.random.Generator(np.random.PCG64(seed))
    if kind == "lognormal":
        return np.exp(g.normal(0.0, 3.0, size=n))
    if kind == "equal":
        return np.ones(n)
    if kind == "dominant":
        w = g.random(n) * 1e-9
        w[g.integers(0, n)] = 1.0
        return w
    if kind == "zeros":
        w = g.random(n)
        w[g.random(n) < 0.5] = 0.0
        if not w.any():
            w[0] = 1.0
        return w
    if kind == "tiny":
        return np.exp(g.uniform(-700.0, 0.0, size=n))
    if kind == "single":
        w = np.zeros(n)
        w[g.integers(0, n)] = g.random() + 0.5
        return w
    raise ValueError(kind)
