// Device models of the nested state space of Section 2, Eq. (1).
//
// Each model is a struct of static device functions over small register
// arrays, split so that the work that depends only on the outer state is
// done once per segment when it is uniform there:
//
//   fx(P, x, z, nu, t, xn)        x_{t+1} = f^x(x_t, z_t, v^x)    (nu: DX normals)
//   fz_pre(P, x, xn, t, pre)      the part of f^z that depends only on x_{t:t+1}
//                                 (and on t, for a time-varying model): NPRE
//                                 values (DZ unless the model says otherwise)
//   fz_post(P, pre, z, nu, zn)    z_{t+1} = f^z(x_{t:t+1}, z_t, v^z) (nu: DZ normals)
//   obs_pre(P, y, x, r0)          the part of y - h(x, z) that depends only on x
//   logpy_post(P, r0, z)          log p(y_t | x_t, z_t)
//   logpx(P, xn, x, z, t)         log p(x_{t+1} | x_t, z_t)
//   px_pre(P, xn, x, t, c)        models whose logpx depends on z (kXdepZ): the
//                                 part that does not, NPX values, so that
//   logpx_post(P, c, z)           gives logpx for many z at the cost of the
//                                 z-dependent terms alone
//   obs_mean(P, x, z, h)          the noise-free observation h(x, z) (models with
//                                 a one-dimensional y: the predicted observation)
//
// t is the time of the state the transition leaves (used only by a
// time-varying model).
//
// kXdepZ says whether p(x_{t+1} | x_t, z_t) depends on z_t; when it does
// not, the x-conditioning factor of eq:qnobar is constant over the inner
// cloud and the kernels skip it.
//
// kStreamZ models (a wide z, y = C z + e with 32 components) give f^z one
// z component at a time, so that a kernel forms z_{t+1} component by
// component and hands each pair to the matrix cores for the residual
// y - C z of a wave's particles at once, and the likelihood as a sum of
// per-component terms:
//   fz_lite(P, x, xn, t, c)       a compact form of fz_pre (NPL values)
//   fz_pre_lite(P, c, k)          pre[k] from it
//   fz_post_k(P, prek, z, nuk, k) component k of fz_post
//   Layout::C                     C, [DY][DZ] row-major
//   row_term(P, e)                the likelihood's term of one residual component
//   logpy_sum(P, s)               log p(y | z) from the sum of the terms
// fz_pre and fz_post are the first three composed, with the same arithmetic
// in the same order; logpy_post(P, y, z) = logpy_sum(sum_k row_term(e_k)).
//
// Parameters live in one float array in device memory (read through Prm): the raw parameter
// values in the interface's blob order, followed by constants the host
// derives from them in double precision (square roots, reciprocals, log
// normalisers) at fixed offsets given by each model's `Layout`.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

namespace dpf {

constexpr float kLn2Pi = 1.8378770664093453f;
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kInv2Pi = 0.15915494309189535f;

// Model parameters are read-only for a whole launch.  Reading them through
// the constant address space lets the compiler use scalar loads for them
// (they are uniform) even after the kernel's own global stores.
using Prm = const __attribute__((address_space(4))) float*;
__device__ __forceinline__ Prm as_prm(const float* p) { return (Prm)p; }

__device__ __forceinline__ float fast_exp(float v) { return __builtin_amdgcn_exp2f(v * kLog2e); }
__device__ __forceinline__ float fast_log(float v) { return __builtin_amdgcn_logf(v) * 0.6931471805599453f; }

// cos a and sin a for an angle in radians that runs to thousands (a drift
// in t): a / 2 pi reduced to [-1/2, 1/2] revolutions in double, then the
// hardware cosine / sine of that many revolutions in FP32 (absolute error of
// order 1e-6; the FP64 library functions cost tens of FP64 instructions).
__device__ __forceinline__ float cos_rad(double a) {
  const double r = a * 0.15915494309189535;
  return __builtin_amdgcn_cosf((float)(r - rint(r)));
}
__device__ __forceinline__ float sin_rad(double a) {
  const double r = a * 0.15915494309189535;
  return __builtin_amdgcn_sinf((float)(r - rint(r)));
}

// tanh(a) = sign(a) (1 - 2 / (exp(2|a|) + 1)); absolute error ~1e-7.
__device__ __forceinline__ float tanh_f(float a) {
  const float e = fast_exp(2.0f * fabsf(a));
  const float r = 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
  return copysignf(r, a);
}

// ---------------------------------------------------------------- LINGAUSS
// x' = Ax x + Cxz z + sqrt(qx) v ; z' = Az z + Bzx x' + sqrt(qz) w ;
// y = Hx x + Hz z + sqrt(r) e.
template <int DX_, int DZ_, int DY_>
struct LinGauss {
  static constexpr int DX = DX_, DZ = DZ_, DY = DY_, NPRE = DZ_;
  static constexpr bool kXdepZ = true;
  static constexpr bool kStreamZ = false;
  struct Layout {
    static constexpr int Ax = 0, Cxz = Ax + DX * DX, qx = Cxz + DX * DZ, Az = qx + 1,
                         Bzx = Az + DZ * DZ, qz = Bzx + DZ * DX, Hx = qz + 1, Hz = Hx + DY * DX,
                         r = Hz + DY * DZ, n_raw = r + 1;
    // derived
    static constexpr int sx = n_raw, sz = sx + 1, inv_qx = sz + 1, inv_r = inv_qx + 1,
                         cx = inv_r + 1, cy = cx + 1, n_total = cy + 1;
  };
  using L = Layout;

  __device__ static void fx(Prm P, const float* x, const float* z, const float* nu, int,
                            float* xn) {
#pragma unroll
    for (int a = 0; a < DX; ++a) {
      float s = 0.f;
#pragma unroll
      for (int b = 0; b < DX; ++b) s += P[L::Ax + a * DX + b] * x[b];
#pragma unroll
      for (int b = 0; b < DZ; ++b) s += P[L::Cxz + a * DZ + b] * z[b];
      xn[a] = s + P[L::sx] * nu[a];
    }
  }
  __device__ static void fz_pre(Prm P, const float* x, const float* xn, int t, float* pre) {
#pragma unroll
    for (int a = 0; a < DZ; ++a) pre[a] = fz_pre_k(P, x, xn, t, a);
  }
  __device__ static float fz_pre_k(Prm P, const float*, const float* xn, int, int a) {
    float s = 0.f;
#pragma unroll
    for (int b = 0; b < DX; ++b) s += P[L::Bzx + a * DX + b] * xn[b];
    return s;
  }
  __device__ static void fz_post(Prm P, const float* pre, const float* z, const float* nu,
                                 float* zn) {
#pragma unroll
    for (int a = 0; a < DZ; ++a) {
      float s = pre[a];
#pragma unroll
      for (int b = 0; b < DZ; ++b) s += P[L::Az + a * DZ + b] * z[b];
      zn[a] = s + P[L::sz] * nu[a];
    }
  }
  __device__ static void obs_pre(Prm P, const float* y, const float* x, float* r0) {
#pragma unroll
    for (int a = 0; a < DY; ++a) {
      float s = y[a];
#pragma unroll
      for (int b = 0; b < DX; ++b) s -= P[L::Hx + a * DX + b] * x[b];
      r0[a] = s;
    }
  }
  __device__ static float logpy_post(Prm P, const float* r0, const float* z) {
    float q = 0.f;
#pragma unroll
    for (int a = 0; a < DY; ++a) {
      float e = r0[a];
#pragma unroll
      for (int b = 0; b < DZ; ++b) e -= P[L::Hz + a * DZ + b] * z[b];
      q += e * e;
    }
    return P[L::cy] - 0.5f * P[L::inv_r] * q;
  }
  // noise-free observation h(x, z) = Hx x + Hz z
  __device__ static void obs_mean(Prm P, const float* x, const float* z, float* h) {
#pragma unroll
    for (int a = 0; a < DY; ++a) {
      float s = 0.f;
#pragma unroll
      for (int b = 0; b < DX; ++b) s += P[L::Hx + a * DX + b] * x[b];
#pragma unroll
      for (int b = 0; b < DZ; ++b) s += P[L::Hz + a * DZ + b] * z[b];
      h[a] = s;
    }
  }
  static constexpr int NPX = DX;
  // x' - Ax x
  __device__ static void px_pre(Prm P, const float* xn, const float* x, int, float* c) {
#pragma unroll
    for (int a = 0; a < DX; ++a) {
      float s = xn[a];
#pragma unroll
      for (int b = 0; b < DX; ++b) s -= P[L::Ax + a * DX + b] * x[b];
      c[a] = s;
    }
  }
  __device__ static float logpx_post(Prm P, const float* c, const float* z) {
    float q = 0.f;
#pragma unroll
    for (int a = 0; a < DX; ++a) {
      float s = c[a];
#pragma unroll
      for (int b = 0; b < DZ; ++b) s -= P[L::Cxz + a * DZ + b] * z[b];
      q += s * s;
    }
    return P[L::cx] - 0.5f * P[L::inv_qx] * q;
  }
  __device__ static float logpx(Prm P, const float* xn, const float* x, const float* z, int t) {
    float c[NPX];
    px_pre(P, xn, x, t, c);
    return logpx_post(P, c, z);
  }
};

// Growth model of the outer block shared by NONLIN and HIGHDIM:
// x'_d = a x_d + b x_d / (1 + x_d^2) + sqrt(qx) v_d.
__device__ __forceinline__ float growth(float a, float b, float x) {
  return a * x + b * x * __builtin_amdgcn_rcpf(1.0f + x * x);
}

// ------------------------------------------------------------------ NONLIN
// z' = tanh(W x') + rho z + sqrt(qz) w ; y_k = z_k + c g_k(x) + sqrt(r) e_k
// with g_k = x_{k mod DX}^2 (bmode 0) or |x|^2 (bmode 1).
template <int DX_, int DZ_>
struct NonLin {
  static constexpr int DX = DX_, DZ = DZ_, DY = DZ_, NPRE = DZ;
  static constexpr bool kXdepZ = false;
  static constexpr bool kStreamZ = false;
  struct Layout {
    static constexpr int a = 0, b = 1, qx = 2, W = 3, rho = W + DZ * DX, qz = rho + 1, c = qz + 1,
                         r = c + 1, bmode = r + 1, n_raw = bmode + 1;
    static constexpr int sx = n_raw, sz = sx + 1, inv_qx = sz + 1, inv_r = inv_qx + 1,
                         cx = inv_r + 1, cy = cx + 1, n_total = cy + 1;
  };
  using L = Layout;

  __device__ static void fx(Prm P, const float* x, const float*, const float* nu, int,
                            float* xn) {
    const float a = P[L::a], b = P[L::b], s = P[L::sx];
#pragma unroll
    for (int d = 0; d < DX; ++d) xn[d] = growth(a, b, x[d]) + s * nu[d];
  }
  __device__ static void fz_pre(Prm P, const float* x, const float* xn, int t, float* pre) {
#pragma unroll
    for (int k = 0; k < DZ; ++k) pre[k] = fz_pre_k(P, x, xn, t, k);
  }
  __device__ static float fz_pre_k(Prm P, const float*, const float* xn, int, int k) {
    float s = 0.f;
#pragma unroll
    for (int d = 0; d < DX; ++d) s += P[L::W + k * DX + d] * xn[d];
    return tanh_f(s);
  }
  __device__ static void fz_post(Prm P, const float* pre, const float* z, const float* nu,
                                 float* zn) {
    const float rho = P[L::rho], s = P[L::sz];
#pragma unroll
    for (int k = 0; k < DZ; ++k) zn[k] = pre[k] + rho * z[k] + s * nu[k];
  }
  __device__ static void obs_pre(Prm P, const float* y, const float* x, float* r0) {
    const float c = P[L::c];
    if (P[L::bmode] == 0.0f) {
#pragma unroll
      for (int k = 0; k < DY; ++k) r0[k] = y[k] - c * x[k % DX] * x[k % DX];
    } else {
      float q = 0.f;
#pragma unroll
      for (int d = 0; d < DX; ++d) q += x[d] * x[d];
#pragma unroll
      for (int k = 0; k < DY; ++k) r0[k] = y[k] - c * q;
    }
  }
  __device__ static float logpy_post(Prm P, const float* r0, const float* z) {
    float q = 0.f;
#pragma unroll
    for (int k = 0; k < DY; ++k) {
      const float e = r0[k] - z[k];
      q += e * e;
    }
    return P[L::cy] - 0.5f * P[L::inv_r] * q;
  }
  __device__ static float logpx(Prm P, const float* xn, const float* x, const float*, int) {
    const float a = P[L::a], b = P[L::b];
    float q = 0.f;
#pragma unroll
    for (int d = 0; d < DX; ++d) {
      const float e = xn[d] - growth(a, b, x[d]);
      q += e * e;
    }
    return P[L::cx] - 0.5f * P[L::inv_qx] * q;
  }
};

// ----------------------------------------------------------------- HIGHDIM
// z' = A z + B sin(x') + sqrt(qz) w with A tridiagonal ; y = C z + e with
// per-component density (1-eps) N(0, r) + eps t_nu(e/sqrt r)/sqrt r.
template <int DX_, int DZ_, int DY_>
struct HighDim {
  static constexpr int DX = DX_, DZ = DZ_, DY = DY_, NPRE = DZ;
  static constexpr bool kXdepZ = false;
  static constexpr bool kStreamZ = true;
  static constexpr int NPL = DX;
  struct Layout {
    static constexpr int a = 0, b = 1, qx = 2, Alo = 3, Adg = Alo + DZ - 1, Aup = Adg + DZ,
                         B = Aup + DZ - 1, qz = B + DZ * DX, C = qz + 1, r = C + DY * DZ,
                         eps = r + 1, nu = eps + 1, gonly = nu + 1, n_raw = gonly + 1;
    // derived: sx sz inv_qx cx ; Gaussian-only: inv_r, cy (all DY components) ;
    // mixture: half_inv_r, lg0 = log(1-eps) - 0.5 log(2 pi r),
    //          lt0 = log eps + lgamma((nu+1)/2) - lgamma(nu/2) - 0.5 log(nu pi r),
    //          tnu = (nu+1)/2, inv_nur = 1/(nu r)
    static constexpr int sx = n_raw, sz = sx + 1, inv_qx = sz + 1, cx = inv_qx + 1,
                         inv_r = cx + 1, cy = inv_r + 1, lg0 = cy + 1, lt0 = lg0 + 1,
                         tnu = lt0 + 1, inv_nur = tnu + 1, n_total = inv_nur + 1;
  };
  using L = Layout;

  __device__ static void fx(Prm P, const float* x, const float*, const float* nu, int,
                            float* xn) {
    const float a = P[L::a], b = P[L::b], s = P[L::sx];
#pragma unroll
    for (int d = 0; d < DX; ++d) xn[d] = growth(a, b, x[d]) + s * nu[d];
  }
  // c = sin(x'); pre[k] = (B sin(x'))_k
  __device__ static void fz_lite(Prm, const float*, const float* xn, int, float* c) {
#pragma unroll
    for (int d = 0; d < DX; ++d) c[d] = __builtin_amdgcn_sinf(xn[d] * kInv2Pi);
  }
  __device__ static float fz_pre_lite(Prm P, const float* c, int k) {
    float s = 0.f;
#pragma unroll
    for (int d = 0; d < DX; ++d) s += P[L::B + k * DX + d] * c[d];
    return s;
  }
  __device__ static void fz_pre(Prm P, const float* x, const float* xn, int t, float* pre) {
    float c[NPL];
    fz_lite(P, x, xn, t, c);
#pragma unroll
    for (int k = 0; k < DZ; ++k) pre[k] = fz_pre_lite(P, c, k);
  }
  __device__ static float fz_pre_k(Prm P, const float* x, const float* xn, int t, int k) {
    float c[NPL];
    fz_lite(P, x, xn, t, c);
    return fz_pre_lite(P, c, k);
  }
  // component k of A z + pre + sqrt(qz) nu, A tridiagonal
  __device__ static float fz_post_k(Prm P, float prek, const float* z, float nuk, int k) {
    float v = prek + P[L::Adg + k] * z[k] + P[L::sz] * nuk;
    if (k > 0) v += P[L::Alo + k - 1] * z[k - 1];
    if (k + 1 < DZ) v += P[L::Aup + k] * z[k + 1];
    return v;
  }
  __device__ static void fz_post(Prm P, const float* pre, const float* z, const float* nu,
                                 float* zn) {
#pragma unroll
    for (int k = 0; k < DZ; ++k) zn[k] = fz_post_k(P, pre[k], z, nu[k], k);
  }
  __device__ static void obs_pre(Prm, const float* y, const float*, float* r0) {
#pragma unroll
    for (int k = 0; k < DY; ++k) r0[k] = y[k];
  }
  // Gaussian: cy - q / (2 r), q the sum of e_k^2; mixture: the sum over the
  // components of log((1 - eps) N(e_k; 0, r) + eps t_nu(e_k; 0, r)), each as
  // max + log(1 + exp(-|difference|))
  __device__ static float row_term(Prm P, float e) {
    const float e2 = e * e;
    if (P[L::gonly] != 0.0f) return e2;
    const float lg = P[L::lg0] - 0.5f * P[L::inv_r] * e2;
    const float lt = P[L::lt0] - P[L::tnu] * fast_log(1.0f + e2 * P[L::inv_nur]);
    const float mx = fmaxf(lg, lt);
    return mx + fast_log(1.0f + fast_exp(-fabsf(lg - lt)));
  }
  __device__ static float logpy_sum(Prm P, float s) {
    return P[L::gonly] != 0.0f ? P[L::cy] - 0.5f * P[L::inv_r] * s : s;
  }
  // one particle on the vector ALU, row by row
  __device__ static float logpy_post(Prm P, const float* r0, const float* z) {
    float s = 0.f;
#pragma unroll 4
    for (int k = 0; k < DY; ++k) {
      float v = r0[k];
#pragma unroll
      for (int d = 0; d < DZ; ++d) v -= P[L::C + k * DZ + d] * z[d];
      s += row_term(P, v);
    }
    return logpy_sum(P, s);
  }
  __device__ static float logpx(Prm P, const float* xn, const float* x, const float*, int) {
    const float a = P[L::a], b = P[L::b];
    float q = 0.f;
#pragma unroll
    for (int d = 0; d < DX; ++d) {
      const float e = xn[d] - growth(a, b, x[d]);
      q += e * e;
    }
    return P[L::cx] - 0.5f * P[L::inv_qx] * q;
  }
};

// ------------------------------------------------------------------ TWODIM
// Model 1 of Table 1 (the 2-dimensional example), dx = dz = dy = 1, in
// either sampling order, with an optional change point.  In the paper's
// variables (x, z):
//   x' = x + z / (1 + z^2) + v^x ,
//   z' = x + rho z + b z / (1 + z^2) + amp cos(freq t) + v^z ,
//   y  = atan(x) + z^2 / 20 + e ,
// (v^x, v^z) ~ N(0, [[qx, cxz], [cxz, qz]]), e ~ N(0, r); t is the time of
// the state the transition leaves.  From t >= tswap on the two transition
// models are swapped (x' = z + rho x + b x / (1 + x^2) + amp cos(freq t) + v^x,
// z' = z + x / (1 + x^2) + v^z; the noises stay with their variables): the
// change point of the decomposition experiment of Section 4.3.
// ZF = false samples x first (outer x, inner z, DPF_MODEL_TWODIM); ZF = true
// samples z first (outer z, inner x, DPF_MODEL_TWODIM_ZFIRST), the other
// action of Section 4.3.  With outer o and inner i, one of them follows the
// "slow" law s' = s + g / (1 + g^2) and the other the "growth" law
// g' = s + rho g + b g / (1 + g^2) + amp cos(freq t); the outer transition
// depends on the inner variable (kXdepZ), and given o' the inner noise is
// v_i | v_o ~ N(k v_o, q_i - cxz^2 / q_o), k = cxz / q_o.  Every form of the
// inner transition is c1 i + c2 i / (1 + i^2) + (terms of o, o', t) + noise,
// so fz_pre passes (terms, c1, c2) and NPRE = 3.
template <bool ZF>
struct Table1M1 {
  static constexpr int DX = 1, DZ = 1, DY = 1, NPRE = 3;
  static constexpr bool kXdepZ = true;
  static constexpr bool kStreamZ = false;
  struct Layout {
    static constexpr int qx = 0, qz = 1, cxz = 2, rho = 3, b = 4, amp = 5, freq = 6, r = 7, tswap = 8,
                         n_raw = 9;
    // so = sqrt(q_o), k = cxz / q_o, sic = sqrt(q_i - cxz^2 / q_o)
    static constexpr int so = n_raw, k = so + 1, sic = k + 1, inv_qo = sic + 1, co = inv_qo + 1,
                         inv_r = co + 1, cy = inv_r + 1, n_total = cy + 1;
  };
  using L = Layout;

  __device__ static float sat(float v) { return v / (1.0f + v * v); }
  __device__ static float cyc(Prm P, int t) { return P[L::amp] * cos_rad((double)P[L::freq] * (double)t); }
  // whether the outer variable follows the slow law at t
  __device__ static bool outer_slow(Prm P, int t) { return ((float)t >= P[L::tswap]) == ZF; }
  __device__ static float mean_o(Prm P, float o, float i, int t) {
    return outer_slow(P, t) ? o + sat(i) : i + P[L::rho] * o + P[L::b] * sat(o) + cyc(P, t);
  }
  __device__ static void fx(Prm P, const float* x, const float* z, const float* nu, int t, float* xn) {
    xn[0] = mean_o(P, x[0], z[0], t) + P[L::so] * nu[0];
  }
  __device__ static void fz_pre(Prm P, const float* x, const float* xn, int t, float* pre) {
    const float o = x[0], on = xn[0], k = P[L::k];
    if (outer_slow(P, t)) {
      // inner growth: o + A + k (o' - o) + rho i + (b - k) sat(i)
      pre[0] = o + cyc(P, t) + k * (on - o);
      pre[1] = P[L::rho];
      pre[2] = P[L::b] - k;
    } else {
      // inner slow: sat(o) + k (o' - rho o - b sat(o) - A) + (1 - k) i
      pre[0] = sat(o) + k * (on - P[L::rho] * o - P[L::b] * sat(o) - cyc(P, t));
      pre[1] = 1.0f - k;
      pre[2] = 0.0f;
    }
  }
  __device__ static void fz_post(Prm P, const float* pre, const float* z, const float* nu, float* zn) {
    zn[0] = pre[1] * z[0] + pre[2] * sat(z[0]) + pre[0] + P[L::sic] * nu[0];
  }
  __device__ static void obs_pre(Prm, const float* y, const float* x, float* r0) {
    r0[0] = ZF ? y[0] - 0.05f * x[0] * x[0] : y[0] - atanf(x[0]);
  }
  __device__ static float logpy_post(Prm P, const float* r0, const float* z) {
    const float e = ZF ? r0[0] - atanf(z[0]) : r0[0] - 0.05f * z[0] * z[0];
    return P[L::cy] - 0.5f * P[L::inv_r] * e * e;
  }
  // x' - mean_o = c0 - c1 i - c2 sat(i)
  static constexpr int NPX = 3;
  __device__ static void px_pre(Prm P, const float* xn, const float* x, int t, float* c) {
    const float o = x[0];
    if (outer_slow(P, t)) {
      c[0] = xn[0] - o;
      c[1] = 0.0f;
      c[2] = 1.0f;
    } else {
      c[0] = xn[0] - (P[L::rho] * o + P[L::b] * sat(o) + cyc(P, t));
      c[1] = 1.0f;
      c[2] = 0.0f;
    }
  }
  __device__ static float logpx_post(Prm P, const float* c, const float* z) {
    // (c[2] is 0 under the growth law of the outer variable: sat(i) is
    // skipped, the same value as multiplying it by 0 for finite i)
    const float si = c[2] != 0.0f ? c[2] * sat(z[0]) : 0.0f;
    const float e = c[0] - c[1] * z[0] - si;
    return P[L::co] - 0.5f * P[L::inv_qo] * e * e;
  }
  __device__ static float logpx(Prm P, const float* xn, const float* x, const float* z, int t) {
    float c[NPX];
    px_pre(P, xn, x, t, c);
    return logpx_post(P, c, z);
  }
  // noise-free observation h(x, z) = atan(x) + z^2 / 20
  __device__ static void obs_mean(Prm, const float* x, const float* z, float* h) {
    h[0] = ZF ? atanf(z[0]) + 0.05f * x[0] * x[0] : atanf(x[0]) + 0.05f * z[0] * z[0];
  }
};
using TwoDim = Table1M1<false>;
using TwoDimZ = Table1M1<true>;

// ----------------------------------------------------------------- FOURDIM
// Model 2 of Table 1 (the 4-dimensional example), dx = dz = 2, dy = 1:
//   x1' = a1 x1 + bs sin t + v1 ,  x2' = c21 x1 + a2 x2 + v2 ,
//   z1' = z1 + z2 / (1 + z2^2) + w1 ,
//   z2' = z1' + rho z2 + b z2 / (1 + z2^2) + amp cos(freq t) + w2 ,
//   y   = (x1 + x2) / (1 + x1^2) + atan(z1) + z2^2 / 20 + e ,
// v ~ N(0, diag(qx1, qx2)), (w1, w2) ~ N(0, [[qz1, cz], [cz, qz2]]) drawn as
// w1 = sqrt(qz1) nu1, w2 = (cz / qz1) w1 + sqrt(qz2 - cz^2 / qz1) nu2, e ~ N(0, r);
// t is the time of the state the transition leaves.  The blocks are coupled
// only through y (p(x' | x, z) does not depend on z).
struct FourDim {
  static constexpr int DX = 2, DZ = 2, DY = 1, NPRE = 2;
  static constexpr bool kXdepZ = false;
  static constexpr bool kStreamZ = false;
  struct Layout {
    static constexpr int a1 = 0, bs = 1, c21 = 2, a2 = 3, qx1 = 4, qx2 = 5, qz1 = 6, qz2 = 7, cz = 8, rho = 9,
                         b = 10, amp = 11, freq = 12, r = 13, n_raw = 14;
    static constexpr int sx1 = n_raw, sx2 = sx1 + 1, sz1 = sx2 + 1, kz = sz1 + 1, szc = kz + 1,
                         inv_qx1 = szc + 1, inv_qx2 = inv_qx1 + 1, cx = inv_qx2 + 1, inv_r = cx + 1,
                         cy = inv_r + 1, n_total = cy + 1;
  };
  using L = Layout;

  __device__ static float drift_x(Prm P, int t) { return P[L::bs] * sin_rad((double)t); }
  __device__ static void fx(Prm P, const float* x, const float*, const float* nu, int t, float* xn) {
    xn[0] = P[L::a1] * x[0] + drift_x(P, t) + P[L::sx1] * nu[0];
    xn[1] = P[L::c21] * x[0] + P[L::a2] * x[1] + P[L::sx2] * nu[1];
  }
  __device__ static float fz_pre_k(Prm P, const float*, const float*, int t, int k) {
    return k == 1 ? P[L::amp] * cos_rad((double)P[L::freq] * (double)t) : 0.0f;
  }
  __device__ static void fz_pre(Prm P, const float* x, const float* xn, int t, float* pre) {
    pre[0] = 0.0f;
    pre[1] = fz_pre_k(P, x, xn, t, 1);
  }
  __device__ static void fz_post(Prm P, const float* pre, const float* z, const float* nu, float* zn) {
    const float g = z[1] / (1.0f + z[1] * z[1]);
    const float w1 = P[L::sz1] * nu[0];
    const float z1 = z[0] + g + w1;
    zn[0] = z1;
    zn[1] = z1 + P[L::rho] * z[1] + P[L::b] * g + pre[1] + P[L::kz] * w1 + P[L::szc] * nu[1];
  }
  __device__ static void obs_pre(Prm, const float* y, const float* x, float* r0) {
    r0[0] = y[0] - (x[0] + x[1]) / (1.0f + x[0] * x[0]);
  }
  __device__ static float logpy_post(Prm P, const float* r0, const float* z) {
    const float e = r0[0] - atanf(z[0]) - 0.05f * z[1] * z[1];
    return P[L::cy] - 0.5f * P[L::inv_r] * e * e;
  }
  // noise-free observation h(x, z) = (x1 + x2) / (1 + x1^2) + atan(z1) + z2^2 / 20
  __device__ static void obs_mean(Prm, const float* x, const float* z, float* h) {
    h[0] = (x[0] + x[1]) / (1.0f + x[0] * x[0]) + atanf(z[0]) + 0.05f * z[1] * z[1];
  }
  __device__ static float logpx(Prm P, const float* xn, const float* x, const float*, int t) {
    const float e0 = xn[0] - (P[L::a1] * x[0] + drift_x(P, t));
    const float e1 = xn[1] - (P[L::c21] * x[0] + P[L::a2] * x[1]);
    return P[L::cx] - 0.5f * (P[L::inv_qx1] * e0 * e0 + P[L::inv_qx2] * e1 * e1);
  }
};

}  // namespace dpf
