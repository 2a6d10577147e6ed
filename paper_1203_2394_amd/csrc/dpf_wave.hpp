// Wave64 cross-lane reductions and scans with DPP (data-parallel primitives).
//
// DPP moves operate inside the vector ALU, so a reduction or scan step costs
// a few cycles instead of an LDS round trip per step.  A wave is handled as
// four rows of 16 lanes:
//   row reduce: quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror,
//               row_mirror -- every lane of the row ends with the row total,
//               combined in the same pairing order in every lane (addition
//               and max are commutative, so all lanes hold identical bits);
//   row scan:   row_shr 1, 2, 4, 8 with zero fill (Hillis-Steele);
//   rows:       row totals read with readlane and combined in a fixed order.
// FP64 values move as two 32-bit halves.  Segments of 16 lanes are rows, of
// 32 lanes two rows; 64 lanes are the whole wave.  Every lane of the wave
// must be active.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

namespace dpf {

// DPP control codes (GFX9 encoding).
constexpr int kDppQuadXor1 = 0xB1;     // quad_perm [1,0,3,2]
constexpr int kDppQuadXor2 = 0x4E;     // quad_perm [2,3,0,1]
constexpr int kDppRowHalfMirror = 0x141;
constexpr int kDppRowMirror = 0x140;
constexpr int kDppRowShr1 = 0x111;
constexpr int kDppRowShr2 = 0x112;
constexpr int kDppRowShr4 = 0x114;
constexpr int kDppRowShr8 = 0x118;

template <int CTRL>
__device__ __forceinline__ int dpp_i(int v, int fill) {
  return __builtin_amdgcn_update_dpp(fill, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v, float fill) {
  return __int_as_float(dpp_i<CTRL>(__float_as_int(v), __float_as_int(fill)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v, double fill) {
  const int lo = dpp_i<CTRL>(__double2loint(v), __double2loint(fill));
  const int hi = dpp_i<CTRL>(__double2hiint(v), __double2hiint(fill));
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ float readlane_f(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ __forceinline__ double readlane_d(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float readlane_of(float v, int lane) { return readlane_f(v, lane); }
__device__ __forceinline__ double readlane_of(double v, int lane) { return readlane_d(v, lane); }

struct OpAdd {
  template <class T>
  __device__ static T apply(T a, T b) { return a + b; }
};
struct OpMax {
  __device__ static float apply(float a, float b) { return fmaxf(a, b); }
  __device__ static double apply(double a, double b) { return fmax(a, b); }
};

template <class Op>
__device__ __forceinline__ float row_reduce(float v) {
  v = Op::apply(v, dpp_f<kDppQuadXor1>(v, v));
  v = Op::apply(v, dpp_f<kDppQuadXor2>(v, v));
  v = Op::apply(v, dpp_f<kDppRowHalfMirror>(v, v));
  v = Op::apply(v, dpp_f<kDppRowMirror>(v, v));
  return v;
}
template <class Op>
__device__ __forceinline__ double row_reduce(double v) {
  v = Op::apply(v, dpp_d<kDppQuadXor1>(v, v));
  v = Op::apply(v, dpp_d<kDppQuadXor2>(v, v));
  v = Op::apply(v, dpp_d<kDppRowHalfMirror>(v, v));
  v = Op::apply(v, dpp_d<kDppRowMirror>(v, v));
  return v;
}

// Reduction over segments of W lanes (W = 16, 32 or 64); every lane of a
// segment gets the segment result.
template <class Op, int W, class T>
__device__ __forceinline__ T seg_reduce_wave(T v) {
  static_assert(W == 16 || W == 32 || W == 64, "segment width");
  v = row_reduce<Op>(v);
  if constexpr (W == 16) {
    return v;
  } else {
    const T r0 = readlane_of(v, 0), r1 = readlane_of(v, 16), r2 = readlane_of(v, 32), r3 = readlane_of(v, 48);
    const int lane = threadIdx.x & 63;
    if constexpr (W == 32) {
      return lane < 32 ? Op::apply(r0, r1) : Op::apply(r2, r3);
    } else {
      return Op::apply(Op::apply(r0, r1), Op::apply(r2, r3));
    }
  }
}

// Inclusive sum scan over segments of W lanes (W = 16, 32 or 64).  Lanes of
// a row combine in Hillis-Steele order, so neighbouring prefixes may differ
// in association (at the rounding level) from a serial sum.
template <int W, class T>
__device__ __forceinline__ T seg_scan_wave(T v) {
  static_assert(W == 16 || W == 32 || W == 64, "segment width");
  const T z = T(0);
  if constexpr (sizeof(T) == 8) {
    v += dpp_d<kDppRowShr1>(v, z);
    v += dpp_d<kDppRowShr2>(v, z);
    v += dpp_d<kDppRowShr4>(v, z);
    v += dpp_d<kDppRowShr8>(v, z);
  } else {
    v += dpp_f<kDppRowShr1>(v, z);
    v += dpp_f<kDppRowShr2>(v, z);
    v += dpp_f<kDppRowShr4>(v, z);
    v += dpp_f<kDppRowShr8>(v, z);
  }
  if constexpr (W == 16) return v;
  const T t0 = readlane_of(v, 15), t1 = readlane_of(v, 31), t2 = readlane_of(v, 47);
  const int row = (threadIdx.x & 63) >> 4;
  if constexpr (W == 32) {
    if (row == 1) v += t0;
    if (row == 3) v += t2;
  } else {
    if (row == 1) v += t0;
    if (row == 2) v += t0 + t1;
    if (row == 3) v += (t0 + t1) + t2;
  }
  return v;
}

}  // namespace dpf
