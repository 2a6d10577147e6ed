// dpf_proj.hpp: the observation residual e = y - C z of a wave's 64 inner
// particles on the matrix cores, for the wide-z models (kStreamZ: y of 32
// components, z of an even number).
//
// For one outer particle the residuals of its inner particles are a dense
// product, [32 x dz] C times [dz x M] Z.  v_mfma_f32_32x32x2_f32 adds
// A[32][2] B[2][32] to a 32 x 32 FP32 accumulator; here A holds two columns
// of -C, B the same two components of 32 particles' z, and the accumulator
// the residuals of those 32 particles.  Operand lanes: A[i][k] at lane
// i + 32 k, B[k][j] at lane j + 32 k; D[i][j] at lane j + 32 ((i / 4) % 2),
// register (i % 4) + 4 (i / 8).
//
// Lane l of the wave holds inner particle l; the two halves of the wave
// (particles 0-31 and 32-63) have an accumulator each.  For components
// (2s, 2s+1) every lane has its own z_2s and z_2s+1; one v_permlane32_swap
// (the upper half of its first operand exchanged with the lower half of its
// second) turns them into the B operands of both halves.  C never leaves the
// registers: each lane keeps its DZ / 2 values of -C (one per instruction).
//
// After the last component, particle l's 32 residuals lie in two lanes (l
// and l ^ 32, 16 each); each lane sums the likelihood terms of its 16 (in
// register order), a second swap brings the two partial sums of a particle
// together, and the lower half's partial is added first.  A particle's
// result depends only on its own z (and C, y), not on its lane or the other
// particles, so every kernel that uses this gets the same bits for it.
//
// All 64 lanes take part: callers use it from converged code, with zeros in
// the z of lanes that hold no particle (their results are discarded).
#pragma once
#include <hip/hip_runtime.h>

#include "dpf_models.hpp"

namespace dpf {

typedef float f32x16 __attribute__((ext_vector_type(16)));

template <class Mdl>
struct WaveProj {
  static_assert(Mdl::DY == 32 && Mdl::DZ % 2 == 0, "matrix-core residual: 32 observation components, even dz");
  static constexpr int NA = Mdl::DZ / 2;  // instructions per residual (A values per lane)
  f32x16 d0, d1;

  // A operand of instruction s: -C[l % 32][2 s + l / 32]
  static __device__ __forceinline__ void load_a(Prm P, float* ca) {
    const int l = threadIdx.x & 63;
    const int row = l & 31, half = l >> 5;
#pragma unroll
    for (int s = 0; s < NA; ++s) ca[s] = -P[Mdl::Layout::C + row * Mdl::DZ + 2 * s + half];
  }

  __device__ __forceinline__ void start() {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      d0[r] = 0.f;
      d1[r] = 0.f;
    }
  }

  // components 2s and 2s + 1 of every lane's z; a = ca[s]
  __device__ __forceinline__ void add(float a, float z0, float z1) {
    const auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(z0), __float_as_uint(z1), false, false);
    d0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, __uint_as_float(b[0]), d0, 0, 0, 0);
    d1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, __uint_as_float(b[1]), d1, 0, 0, 0);
  }

  // log p(y | z) of this lane's particle; y the observation (DY values in
  // memory), added to -C z row by row.
  __device__ __forceinline__ float logpy(Prm P, const float* y) const {
    const int half = (threadIdx.x >> 5) & 1;
    float s0 = 0.f, s1 = 0.f;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float yi = y[8 * (r >> 2) + 4 * half + (r & 3)];
      s0 += Mdl::row_term(P, yi + d0[r]);
      s1 += Mdl::row_term(P, yi + d1[r]);
    }
    const auto t = __builtin_amdgcn_permlane32_swap(__float_as_uint(s0), __float_as_uint(s1), false, false);
    return Mdl::logpy_sum(P, __uint_as_float(t[0]) + __uint_as_float(t[1]));
  }
};

}  // namespace dpf
