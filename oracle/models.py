"""Nested state-space models of Eq. (1), oracle side (FP64).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Section 2, Eq. (1) writes the model as x_{t+1} = f^x(x_t, z_t, v^x),
z_{t+1} = f^z(x_{t:t+1}, z_t, v^z), y_t = h(x_t, z_t, e_t), equivalently as
p(x_0), p(z_0|x_0), p(x_{t+1}|x_t,z_t), p(z_{t+1}|x_{t:t+1},z_t) and
p(y_t|x_t,z_t), with all parameters known.  Each model below provides

    fx(x, z, nu, t)     sample of x_{t+1} given standard normals nu (dx)
    fz(x, xn, z, nu, t) sample of z_{t+1} given x_t, x_{t+1}, z_t, normals (dz)
    logpx(xn, x, z, t)  log p(x_{t+1} | x_t, z_t)
    (t is the time of the state the transition leaves; only the models of
    Table 1 use it)
    logpy(y, x, z)      log p(y_t | x_t, z_t)

on arrays whose last axis is the state dimension (leading axes broadcast).
The prior is [x_0; z_0] ~ N(0, I) for every model (as in Table 1).

Parameters arrive as the flat float64 blob of the library interface; the
layouts are parsed here, independently of the HIP side:

LINGAUSS (linear-Gaussian; the coupled variant has Cxz != 0):
    Ax[dx*dx] Cxz[dx*dz] qx Az[dz*dz] Bzx[dz*dx] qz Hx[dy*dx] Hz[dy*dz] r
    x' = Ax x + Cxz z + sqrt(qx) v,  z' = Az z + Bzx x' + sqrt(qz) w,
    y  = Hx x + Hz z + sqrt(r) e.
NONLIN (dy = dz):
    a b qx W[dz*dx] rho qz c r bmode
    x'_d = a x_d + b x_d/(1+x_d^2) + sqrt(qx) v_d,
    z'   = tanh(W x') + rho z + sqrt(qz) w,
    y_k  = z_k + c g_k(x) + sqrt(r) e_k,  g_k = x_{k mod dx}^2 (bmode 0)
                                          or |x|^2 (bmode 1).
HIGHDIM:
    a b qx Alo[dz-1] Adiag[dz] Aup[dz-1] B[dz*dx] qz C[dy*dz] r eps nu gonly
    x' as NONLIN's x (dx components),  z' = A z + B sin(x') + sqrt(qz) w with
    A tridiagonal,  y = C z + e where each e_k has density
    (1-eps) N(0, r) + eps * t_nu(e/sqrt(r))/sqrt(r)  (gonly=1: pure N(0, r)).
TWODIM (model 1 of Table 1, dx = dz = dy = 1; TWODIM_ZFIRST: the same
model with z sampled first, outer z and inner x):
    qx qz cxz rho b amp freq r tswap
    x' = x + z/(1+z^2) + v^x,  z' = x + rho z + b z/(1+z^2) + amp cos(freq t) + v^z,
    (v^x, v^z) ~ N(0, [[qx, cxz], [cxz, qz]]),  y = atan(x) + z^2/20 + e, e ~ N(0, r).
    In the factorisation of Eq. (1) the inner transition is conditioned on
    x_{t+1}, i.e. on v^x: v^z | v^x ~ N(cxz/qx v^x, qz - cxz^2/qx).
FOURDIM (model 2 of Table 1, dx = dz = 2, dy = 1):
    a1 bs c21 a2 qx1 qx2 qz1 qz2 cz rho b amp freq r
    x1' = a1 x1 + bs sin t + v1,  x2' = c21 x1 + a2 x2 + v2,
    z1' = z1 + z2/(1+z2^2) + w1,  z2' = z1' + rho z2 + b z2/(1+z2^2) + amp cos(freq t) + w2,
    (v1, v2) ~ N(0, diag(qx1, qx2)), (w1, w2) ~ N(0, [[qz1, cz], [cz, qz2]]),
    y = (x1 + x2)/(1 + x1^2) + atan(z1) + z2^2/20 + e, e ~ N(0, r).
"""
import math

import numpy as np

LINGAUSS, NONLIN, HIGHDIM, TWODIM, FOURDIM, TWODIM_ZFIRST = 1, 2, 3, 4, 5, 6

LOG2PI = math.log(2.0 * math.pi)


def _take(blob, pos, n):
    return np.asarray(blob[pos:pos + n], dtype=np.float64), pos + n


def _matvec(Mat, v):
    """Mat (r, c) times v (..., c) -> (..., r)."""
    return np.einsum("rc,...c->...r", Mat, v)


def _gauss_iso_logpdf(resid, var):
    """log N(resid; 0, var I) summed over the last axis."""
    d = resid.shape[-1]
    return -0.5 * np.sum(resid * resid, axis=-1) / var - 0.5 * d * (LOG2PI + math.log(var))


class LinGauss:
    kind = LINGAUSS

    def __init__(self, dx, dz, dy, blob):
        self.dx, self.dz, self.dy = dx, dz, dy
        p = 0
        a, p = _take(blob, p, dx * dx); self.Ax = a.reshape(dx, dx)
        a, p = _take(blob, p, dx * dz); self.Cxz = a.reshape(dx, dz)
        self.qx = float(blob[p]); p += 1
        a, p = _take(blob, p, dz * dz); self.Az = a.reshape(dz, dz)
        a, p = _take(blob, p, dz * dx); self.Bzx = a.reshape(dz, dx)
        self.qz = float(blob[p]); p += 1
        a, p = _take(blob, p, dy * dx); self.Hx = a.reshape(dy, dx)
        a, p = _take(blob, p, dy * dz); self.Hz = a.reshape(dy, dz)
        self.r = float(blob[p]); p += 1
        if p != len(blob):
            raise ValueError("LINGAUSS blob has %d values, expected %d" % (len(blob), p))

    def mean_x(self, x, z):
        return _matvec(self.Ax, x) + _matvec(self.Cxz, z)

    def fx(self, x, z, nu, t=0):
        return self.mean_x(x, z) + math.sqrt(self.qx) * nu

    def fz(self, x, xn, z, nu, t=0):
        return _matvec(self.Az, z) + _matvec(self.Bzx, xn) + math.sqrt(self.qz) * nu

    def logpx(self, xn, x, z, t=0):
        return _gauss_iso_logpdf(xn - self.mean_x(x, z), self.qx)

    def obs_mean(self, x, z):
        """Noise-free observation Hx x + Hz z."""
        return _matvec(self.Hx, x) + _matvec(self.Hz, z)

    def logpy(self, y, x, z):
        return _gauss_iso_logpdf(y - _matvec(self.Hx, x) - _matvec(self.Hz, z), self.r)


def _growth(a, b, x):
    return a * x + b * x / (1.0 + x * x)


class NonLin:
    kind = NONLIN

    def __init__(self, dx, dz, dy, blob):
        if dy != dz:
            raise ValueError("NONLIN needs dy == dz")
        self.dx, self.dz, self.dy = dx, dz, dy
        self.a, self.b, self.qx = (float(v) for v in blob[0:3])
        p = 3
        a, p = _take(blob, p, dz * dx); self.W = a.reshape(dz, dx)
        self.rho, self.qz, self.c, self.r, bmode = (float(v) for v in blob[p:p + 5])
        p += 5
        self.bmode = int(bmode)
        if p != len(blob):
            raise ValueError("NONLIN blob has %d values, expected %d" % (len(blob), p))

    def fx(self, x, z, nu, t=0):
        return _growth(self.a, self.b, x) + math.sqrt(self.qx) * nu

    def fz(self, x, xn, z, nu, t=0):
        return np.tanh(_matvec(self.W, xn)) + self.rho * z + math.sqrt(self.qz) * nu

    def logpx(self, xn, x, z, t=0):
        return _gauss_iso_logpdf(xn - _growth(self.a, self.b, x), self.qx)

    def obs_offset(self, x):
        """c * g(x) broadcast to the dy outputs."""
        if self.bmode == 0:
            idx = np.arange(self.dy) % self.dx
            return self.c * (x[..., idx] ** 2)
        return self.c * np.sum(x * x, axis=-1, keepdims=True) * np.ones(self.dy)

    def logpy(self, y, x, z):
        return _gauss_iso_logpdf(y - z - self.obs_offset(x), self.r)


class HighDim:
    kind = HIGHDIM

    def __init__(self, dx, dz, dy, blob):
        self.dx, self.dz, self.dy = dx, dz, dy
        self.a, self.b, self.qx = (float(v) for v in blob[0:3])
        p = 3
        lo, p = _take(blob, p, dz - 1)
        dg, p = _take(blob, p, dz)
        up, p = _take(blob, p, dz - 1)
        self.A = np.diag(dg) + np.diag(lo, -1) + np.diag(up, 1)
        a, p = _take(blob, p, dz * dx); self.B = a.reshape(dz, dx)
        self.qz = float(blob[p]); p += 1
        a, p = _take(blob, p, dy * dz); self.C = a.reshape(dy, dz)
        self.r, self.eps, self.nu, gonly = (float(v) for v in blob[p:p + 4])
        p += 4
        self.gaussian_only = bool(gonly)
        if p != len(blob):
            raise ValueError("HIGHDIM blob has %d values, expected %d" % (len(blob), p))

    def fx(self, x, z, nu, t=0):
        return _growth(self.a, self.b, x) + math.sqrt(self.qx) * nu

    def fz(self, x, xn, z, nu, t=0):
        return _matvec(self.A, z) + _matvec(self.B, np.sin(xn)) + math.sqrt(self.qz) * nu

    def logpx(self, xn, x, z, t=0):
        return _gauss_iso_logpdf(xn - _growth(self.a, self.b, x), self.qx)

    def logpy(self, y, x, z):
        e = y - _matvec(self.C, z)
        if self.gaussian_only:
            return _gauss_iso_logpdf(e, self.r)
        sd = math.sqrt(self.r)
        log_g = -0.5 * e * e / self.r - 0.5 * (LOG2PI + math.log(self.r))
        nu = self.nu
        # Student-t density with nu degrees of freedom, scaled by sd.
        log_t_norm = (math.lgamma(0.5 * (nu + 1.0)) - math.lgamma(0.5 * nu)
                      - 0.5 * math.log(nu * math.pi))
        s = e / sd
        log_t = log_t_norm - 0.5 * (nu + 1.0) * np.log1p(s * s / nu) - math.log(sd)
        comp = np.logaddexp(math.log1p(-self.eps) + log_g, math.log(self.eps) + log_t)
        return np.sum(comp, axis=-1)


class TwoDim:
    """Model 1 of Table 1: a scalar outer state driven by the inner one
    (x' depends on z), a time-varying inner drift and correlated noises.

    From t >= tswap on the two transition laws are swapped (x follows the
    law z had and z the law x had; each keeps its own noise): the change
    point of Section 4.3.  zfirst: the decomposition that samples z first,
    i.e. the outer state is z and the inner one x (the other action of
    Section 4.3); the arrays passed in are then (outer z, inner x).
    """
    kind = TWODIM

    def __init__(self, dx, dz, dy, blob, zfirst=False):
        if (dx, dz, dy) != (1, 1, 1):
            raise ValueError("TWODIM is (1, 1, 1)")
        if len(blob) != 9:
            raise ValueError("TWODIM blob has %d values, expected 9" % len(blob))
        self.dx = self.dz = self.dy = 1
        (self.qx, self.qz, self.cxz, self.rho, self.b, self.amp, self.freq, self.r,
         self.tswap) = (float(v) for v in blob)
        self.zfirst = bool(zfirst)
        if zfirst:
            self.kind = TWODIM_ZFIRST

    @staticmethod
    def _sat(v):
        return v / (1.0 + v * v)

    # the two laws in the paper's variables (x, z)
    def _slow(self, s, other):
        return s + self._sat(other)

    def _grow(self, g, other, t):
        return other + self.rho * g + self.b * self._sat(g) + self.amp * math.cos(self.freq * t)

    def _mean_x(self, x, z, t):
        return self._grow(x, z, t) if t >= self.tswap else self._slow(x, z)

    def _mean_z(self, x, z, t):
        return self._slow(z, x) if t >= self.tswap else self._grow(z, x, t)

    def _roles(self):
        """(variance of the outer noise, of the inner one) and the regression
        of the inner noise on the outer one."""
        qo, qi = (self.qz, self.qx) if self.zfirst else (self.qx, self.qz)
        return qo, qi, self.cxz / qo, qi - self.cxz * self.cxz / qo

    def _xz(self, o, i):
        return (i, o) if self.zfirst else (o, i)

    def _mean_o(self, o, i, t):
        x, z = self._xz(o, i)
        return self._mean_z(x, z, t) if self.zfirst else self._mean_x(x, z, t)

    def _mean_i(self, o, i, t):
        x, z = self._xz(o, i)
        return self._mean_x(x, z, t) if self.zfirst else self._mean_z(x, z, t)

    def fx(self, x, z, nu, t=0):
        qo, _, _, _ = self._roles()
        return self._mean_o(x, z, t) + math.sqrt(qo) * nu

    def fz(self, x, xn, z, nu, t=0):
        """Inner transition given the outer one: v_i | v_o ~ N(k v_o, q_i|o)."""
        _, _, k, qc = self._roles()
        vo = xn - self._mean_o(x, z, t)
        return self._mean_i(x, z, t) + k * vo + math.sqrt(qc) * nu

    def logpx(self, xn, x, z, t=0):
        qo, _, _, _ = self._roles()
        return _gauss_iso_logpdf(xn - self._mean_o(x, z, t), qo)

    def obs_mean(self, x, z):
        """Noise-free observation atan(x) + z^2 / 20 (paper variables)."""
        xx, zz = self._xz(x, z)
        return np.arctan(xx) + zz * zz / 20.0

    def logpy(self, y, x, z):
        return _gauss_iso_logpdf(y - self.obs_mean(x, z), self.r)


class FourDim:
    """Model 2 of Table 1: two outer and two inner components coupled only
    through the observation; a sin t drift in x1, a cos(1.2 t) drift in z2,
    correlated inner noises, z2' driven by the new z1'."""
    kind = FOURDIM

    def __init__(self, dx, dz, dy, blob):
        if (dx, dz, dy) != (2, 2, 1):
            raise ValueError("FOURDIM is (2, 2, 1)")
        if len(blob) != 14:
            raise ValueError("FOURDIM blob has %d values, expected 14" % len(blob))
        self.dx, self.dz, self.dy = 2, 2, 1
        (self.a1, self.bs, self.c21, self.a2, self.qx1, self.qx2, self.qz1, self.qz2, self.cz, self.rho,
         self.b, self.amp, self.freq, self.r) = (float(v) for v in blob)
        # (w1, w2) = L (nu1, nu2) with L L^T the inner noise covariance
        self.L = np.linalg.cholesky(np.array([[self.qz1, self.cz], [self.cz, self.qz2]]))

    def mean_x(self, x, t):
        m1 = self.a1 * x[..., 0] + self.bs * math.sin(t)
        m2 = self.c21 * x[..., 0] + self.a2 * x[..., 1]
        return np.stack([m1, m2], axis=-1)

    def fx(self, x, z, nu, t=0):
        return self.mean_x(x, t) + np.sqrt([self.qx1, self.qx2]) * nu

    def fz(self, x, xn, z, nu, t=0):
        w = _matvec(self.L, nu)
        z1 = z[..., 0] + z[..., 1] / (1.0 + z[..., 1] ** 2) + w[..., 0]
        z2 = (z1 + self.rho * z[..., 1] + self.b * z[..., 1] / (1.0 + z[..., 1] ** 2)
              + self.amp * math.cos(self.freq * t) + w[..., 1])
        return np.stack([z1, z2], axis=-1)

    def logpx(self, xn, x, z, t=0):
        e = xn - self.mean_x(x, t)
        return (-0.5 * e[..., 0] ** 2 / self.qx1 - 0.5 * e[..., 1] ** 2 / self.qx2
                - 0.5 * (2 * LOG2PI + math.log(self.qx1) + math.log(self.qx2)))

    def obs_mean(self, x, z):
        """Noise-free observation (x1 + x2)/(1 + x1^2) + atan(z1) + z2^2/20."""
        h = (x[..., 0] + x[..., 1]) / (1.0 + x[..., 0] ** 2) + np.arctan(z[..., 0]) + z[..., 1] ** 2 / 20.0
        return h[..., None]

    def logpy(self, y, x, z):
        h = (x[..., 0] + x[..., 1]) / (1.0 + x[..., 0] ** 2) + np.arctan(z[..., 0]) + z[..., 1] ** 2 / 20.0
        return _gauss_iso_logpdf(y - h[..., None], self.r)


def make_model(kind, dx, dz, dy, blob):
    blob = np.asarray(blob, dtype=np.float64)
    if kind == LINGAUSS:
        return LinGauss(dx, dz, dy, blob)
    if kind == NONLIN:
        return NonLin(dx, dz, dy, blob)
    if kind == HIGHDIM:
        return HighDim(dx, dz, dy, blob)
    if kind == TWODIM:
        return TwoDim(dx, dz, dy, blob)
    if kind == TWODIM_ZFIRST:
        return TwoDim(dx, dz, dy, blob, zfirst=True)
    if kind == FOURDIM:
        return FourDim(dx, dz, dy, blob)
    raise ValueError("unknown model kind %r" % (kind,))
