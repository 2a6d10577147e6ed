// Rao-Blackwellised estimate of the new outer state after a look-ahead step:
// the expectation of the particle that Fig. 4 steps 3-4 produce, given the
// look-ahead pass,
//
//   xhat_rb = sum_i Wbar_i sum_j pi_ij xla^{(i,j)},
//   Wbar = softmax_i log w_i (eq:weightsMC),  pi_i. = softmax_j ell_ij,
//
// instead of the plain mean of the N particles drawn by outer resampling and
// the candidate SIR.  Computed on request from the buffers the step leaves:
// the weights ell and log w of the step, the state it started from (the
// other state copy) and the look-ahead candidates, regenerated from their
// LA_X normals at (t, i, j) exactly as the weights kernel drew them.
//
//   k_rb_outer    one wave per outer particle i: sum_j pi_ij xla^{(i,j)}
//                 (FP64, a row without a finite ell weighs its candidates
//                 uniformly)
//   k_rb_finish   one workgroup per filter: the Wbar-weighted sum (FP64, a
//                 filter without a finite log w weighs uniformly); filters
//                 that did not take the last step get NaN
#pragma once
#include <hip/hip_runtime.h>

#include "dpf_kernels.hpp"
#include "dpf_learned.hpp"

namespace dpf {

template <class Mdl>
__global__ __launch_bounds__(kBlock) void k_rb_outer(StepArgs a, double* xrb) {
  constexpr int DX = Mdl::DX, DZ = Mdl::DZ;
  const int g = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (g >= a.NT) return;  // whole waves
  const int f = filter_of_outer(a.ooff, a.n_filters, g);
  if (!a.act[f]) return;
  const int oo = a.ooff[f], M = a.fM[f];
  const long long io = a.ioff[f];
  const int i = g - oo;
  const int t = a.tcur[f];  // the step just taken
  const unsigned char cb = a.cur[f];
  const int src = copy_of(cb) ^ 1;  // the state the step started from
  const int ci = ident_slots(cb, src) ? i : a.ind[src][oo + i];
  const Key key = make_key(a.seed, (uint32_t)f);
  float x[DX];
#pragma unroll
  for (int d = 0; d < DX; ++d) x[d] = a.x[src][(long long)d * a.NT + g];
  const float* zrow = a.z[src] + (io + (long long)ci * M) * DZ;
  const float* erow = a.ell + io + (long long)i * M;
  const float lse = a.logw[g];
  const bool deg = !finitef(lse);
  double acc[DX];
#pragma unroll
  for (int d = 0; d < DX; ++d) acc[d] = 0.0;
  for (int j = lane; j < M; j += kWave) {
    const float e = erow[j];
    const double w = deg ? 1.0 / M : (finitef(e) ? exp((double)e - (double)lse) : 0.0);
    float z[DZ], nu[DX], xl[DX];
#pragma unroll
    for (int d = 0; d < DZ; ++d) z[d] = zrow[d * M + j];
    normals<DX>(key, (uint32_t)t, (uint32_t)i, (uint32_t)j, P_LA_X, nu);
    Mdl::fx(as_prm(a.prm), x, z, nu, t - 1, xl);
#pragma unroll
    for (int d = 0; d < DX; ++d) acc[d] += w * (double)xl[d];
  }
#pragma unroll
  for (int d = 0; d < DX; ++d) {
    const double s = seg_reduce_wave<OpAdd, kWave>(acc[d]);
    if (lane == 0) xrb[(long long)g * DX + d] = s;
  }
}

template <int DX>
__global__ __launch_bounds__(kBlock) void k_rb_finish(StepArgs a, const double* xrb, float* out) {
  __shared__ float fred4[kBlock / kWave];
  __shared__ double red4[kBlock / kWave];
  const int f = blockIdx.x;
  if (!a.act[f]) {
    if (threadIdx.x < DX) out[f * DX + threadIdx.x] = __builtin_nanf("");
    return;
  }
  const int N = a.fN[f], oo = a.ooff[f];
  float m = -INFINITY;
  for (int i = threadIdx.x; i < N; i += kBlock) {
    const float v = a.logw[oo + i];
    if (finitef(v)) m = fmaxf(m, v);
  }
  m = block_max_256(m, fred4);
  const bool deg = !(m > -INFINITY);
  double s = 0.0, v[DX];
#pragma unroll
  for (int d = 0; d < DX; ++d) v[d] = 0.0;
  for (int i = threadIdx.x; i < N; i += kBlock) {
    const float lw = a.logw[oo + i];
    const double w = deg ? 1.0 : (finitef(lw) ? exp((double)lw - (double)m) : 0.0);
    s += w;
#pragma unroll
    for (int d = 0; d < DX; ++d) v[d] += w * xrb[(long long)(oo + i) * DX + d];
  }
  s = block_sum_256(s, red4);
#pragma unroll
  for (int d = 0; d < DX; ++d) {
    const double vd = block_sum_256(v[d], red4);
    if (threadIdx.x == 0) out[f * DX + d] = (float)(vd / s);
  }
}

}  // namespace dpf
