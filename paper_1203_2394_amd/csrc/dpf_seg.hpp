// Segment primitives for 256-thread workgroups on wave64 hardware.
//
// A workgroup is split into 256/SEG segments of SEG lanes (SEG in
// {16, 32, 64, 128, 256}); one segment serves one outer particle's inner cloud
// of M <= SEG*JPT inner particles, lane l handling inner indices
// l, l+SEG, ... (coalesced in the [N][dz][M] layout).  Segments of up to 64
// lanes live inside one wavefront and reduce / scan with cross-lane
// shuffles; wider segments combine per-wave results through LDS.
//
// Every function here must be reached by all 256 threads (they may contain
// barriers); lanes with nothing to contribute pass the identity.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "dpf_wave.hpp"

namespace dpf {

constexpr int kBlock = 256;
constexpr int kWave = 64;

// Shared scratch for cross-wave combination: one slot per wave (and a spare
// set so that two consecutive primitives do not race).
struct SegScratch {
  float f[2][kBlock / kWave];
  double d[2][kBlock / kWave];
};

template <int SEG>
constexpr int wave_width() { return SEG < kWave ? SEG : kWave; }

template <class Op, int SEG, class T>
__device__ __forceinline__ T seg_reduce(T v, T* red /* [kBlock / kWave] */) {
  v = seg_reduce_wave<Op, wave_width<SEG>()>(v);
  if constexpr (SEG > kWave) {
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) red[w] = v;
    __syncthreads();
    const int w0 = (threadIdx.x / SEG) * (SEG / kWave);
    T r = red[w0];
#pragma unroll
    for (int q = 1; q < SEG / kWave; ++q) r = Op::apply(r, red[w0 + q]);
    __syncthreads();
    v = r;
  }
  return v;
}

// Orders a segment's LDS writes before its reads: a workgroup barrier when
// the segment spans waves, else a wave-level fence (segments in one wave do
// not wait for the other waves of the workgroup).
template <int SEG>
__device__ __forceinline__ void seg_lds_sync() {
  if constexpr (SEG > kWave) {
    __syncthreads();
  } else {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

template <int SEG>
__device__ __forceinline__ float seg_max(float v, SegScratch& sh) {
  return seg_reduce<OpMax, SEG>(v, sh.f[0]);
}

template <int SEG>
__device__ __forceinline__ float seg_sum(float v, SegScratch& sh) {
  return seg_reduce<OpAdd, SEG>(v, sh.f[1]);
}

template <int SEG>
__device__ __forceinline__ double seg_sum_d(double v, SegScratch& sh) {
  return seg_reduce<OpAdd, SEG>(v, sh.d[1]);
}

// Sums of NV values over the segment with one LDS exchange for all of them
// (segments wider than a wavefront).  The result is valid in the segment's
// first lane only.  red: [kBlock / kWave][NV] floats of LDS.
template <int SEG, int NV>
__device__ __forceinline__ void seg_sum_vec(float* v, float (*red)[NV]) {
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = seg_reduce_wave<OpAdd, wave_width<SEG>()>(v[q]);
  if constexpr (SEG > kWave) {
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
#pragma unroll
      for (int q = 0; q < NV; ++q) red[w][q] = v[q];
    }
    __syncthreads();
    if ((threadIdx.x % SEG) == 0) {
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        float r = red[w][q];
#pragma unroll
        for (int qq = 1; qq < SEG / kWave; ++qq) r += red[w + qq][q];
        v[q] = r;
      }
    }
    __syncthreads();
  }
}

// Transpose reduction of NV values (NV a power of two, at most 16) over the
// segment.  Each in-row step pairs lane i with a partner of the same history
// -- row mirror (15 - i), half-row mirror, quad reversal, quad swap, which
// split on lane bits 3, 2, 1, 0 -- and exchanges half of the values still
// held, so a lane adds NV/2 + NV/4 + ... values instead of NV per step; after
// the four steps lane i holds its row's total of slot (i & 15) >> (4 - P)
// (NV = 2^P).  Rows, then waves (through red), are combined in a fixed order.
// Returns the segment total of value `slot` in the lanes that own one
// (slot = -1 elsewhere): lanes 0, 2^(4-P), ... of the segment's first row
// (SEG <= 64), lanes 0..NV-1 of the segment (SEG > 64).
template <int NV>
constexpr int log2_nv() { return NV == 1 ? 0 : NV == 2 ? 1 : NV == 4 ? 2 : NV == 8 ? 3 : 4; }

template <int CTRL, int BIT, int H>
__device__ __forceinline__ void tr_step(float* v, int lane) {
  if constexpr (H == 0) {
    v[0] += dpp_f<CTRL>(v[0], v[0]);
  } else {
    const bool up = (lane >> BIT) & 1;
#pragma unroll
    for (int q = 0; q < H; ++q) {
      const float lo = v[q], hi = v[q + H];
      const float send = up ? lo : hi;
      const float keep = up ? hi : lo;
      v[q] = keep + dpp_f<CTRL>(send, send);
    }
  }
}

template <int SEG, int NV>
__device__ __forceinline__ float seg_sum_vec_t(const float* vin, float (*red)[NV], int& slot) {
  static_assert(NV == 1 || NV == 2 || NV == 4 || NV == 8 || NV == 16, "NV must be a power of two <= 16");
  constexpr int P = log2_nv<NV>();
  constexpr int SH = 4 - P;  // owner lanes are multiples of 2^SH within the row
  float v[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = vin[q];
  const int lane = threadIdx.x & (kWave - 1);
  tr_step<kDppRowMirror, 3, (P >= 1 ? NV / 2 : 0)>(v, lane);
  tr_step<kDppRowHalfMirror, 2, (P >= 2 ? NV / 4 : 0)>(v, lane);
  tr_step<0x1B, 1, (P >= 3 ? NV / 8 : 0)>(v, lane);  // quad_perm [3,2,1,0]
  tr_step<kDppQuadXor1, 0, (P >= 4 ? NV / 16 : 0)>(v, lane);
  float r = v[0];
  constexpr int W = SEG < kWave ? SEG : kWave;
  if constexpr (W >= 32) r += __shfl_xor(r, 16);
  if constexpr (W >= 64) r += __shfl_xor(r, 32);
  const int ls = threadIdx.x % SEG;
  if constexpr (SEG <= kWave) {
    slot = (ls < 16 && (ls & ((1 << SH) - 1)) == 0) ? (ls >> SH) : -1;
    return r;
  } else {
    const int w = threadIdx.x / kWave;
    if (lane < 16 && (lane & ((1 << SH) - 1)) == 0) red[w][lane >> SH] = r;
    __syncthreads();
    float t = 0.f;
    slot = -1;
    if (ls < NV) {
      const int w0 = (threadIdx.x / SEG) * (SEG / kWave);
#pragma unroll
      for (int q = 0; q < SEG / kWave; ++q) t += red[w0 + q][ls];
      slot = ls;
    }
    __syncthreads();
    return t;
  }
}

// For lanes that own a slot of seg_sum_vec_t<SEG, NV>: the total of slot
// `want` (0 <= want < NV; other lanes pass want < 0 and get their own value).
template <int SEG, int NV>
__device__ __forceinline__ float seg_vec_fetch(float tot, int want) {
  constexpr int SH = 4 - log2_nv<NV>();
  const int lane = threadIdx.x & (kWave - 1);
  int src = lane;
  if (want >= 0) {
    if constexpr (SEG <= kWave) {
      const int base = lane - (threadIdx.x % SEG);  // first lane of the segment in this wave
      src = base + (want << SH);
    } else {
      src = (lane & ~15) + want;  // owners are lanes 0..NV-1 of the segment's first wave
    }
  }
  return __shfl(tot, src);
}

// Inclusive FP64 scan within the segment; `total` receives the segment sum.
template <int SEG>
__device__ __forceinline__ double seg_scan_incl(double v, SegScratch& sh, double& total) {
  constexpr int W = wave_width<SEG>();
  v = seg_scan_wave<W>(v);
  if constexpr (SEG <= kWave) {
    if constexpr (W == 16) {
      const int row = (threadIdx.x & 63) >> 4;
      const double t0 = readlane_d(v, 15), t1 = readlane_d(v, 31), t2 = readlane_d(v, 47), t3 = readlane_d(v, 63);
      total = row == 0 ? t0 : (row == 1 ? t1 : (row == 2 ? t2 : t3));
    } else if constexpr (W == 32) {
      total = (threadIdx.x & 63) < 32 ? readlane_d(v, 31) : readlane_d(v, 63);
    } else {
      total = readlane_d(v, 63);
    }
  } else {
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == kWave - 1) sh.d[0][w] = v;
    __syncthreads();
    const int w0 = (threadIdx.x / SEG) * (SEG / kWave);
    double pre = 0.0, tot = 0.0;
#pragma unroll
    for (int q = 0; q < SEG / kWave; ++q) {
      const double s = sh.d[0][w0 + q];
      if (w0 + q < w) pre += s;
      tot += s;
    }
    __syncthreads();
    v += pre;
    total = tot;
  }
  return v;
}

// Systematic search rule: the first index with C[i] > P; if rounding put the
// point at or past the total, the first index with C[i] >= C[n-1].  With
// exact cumulative sums this never selects a zero weight; with rounded ones
// only a point within one rounding unit of a boundary can.
__device__ __forceinline__ int cdf_search(const double* C, int n, double P) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (C[mid] > P)
      hi = mid;
    else
      lo = mid + 1;
  }
  if (lo == n) {
    const double tot = C[n - 1];
    lo = 0;
    hi = n - 1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (C[mid] >= tot)
        hi = mid;
      else
        lo = mid + 1;
    }
  }
  return lo;
}

// Point k of n_out systematic points over total C: ((k + u) * C) / n_out,
// evaluated left to right in IEEE double precision (no contraction: the
// multiply follows an add, never the reverse).
__device__ __forceinline__ double sys_point(int k, double u, double total, int n_out) {
  const double a = (double)k + u;
  const double b = a * total;
  // a power-of-two count: b scaled by 2^-e is the correctly rounded b / n_out
  // as well (the same exact value, one rounding), in one instruction
  if ((n_out & (n_out - 1)) == 0) return __builtin_amdgcn_ldexp(b, -__builtin_ctz((unsigned)n_out));
  return b / (double)n_out;
}

__device__ __forceinline__ bool finitef(float v) { return fabsf(v) <= 3.402823466e38f; }

}  // namespace dpf
