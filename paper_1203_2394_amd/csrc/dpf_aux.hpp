// Small service kernels: per-filter reset, activity mask for multi-step
// runs, state export / import, and the kernel-level primitives exposed for
// testing (raw Philox words, normals, systematic resampling) -- the latter
// call the same device functions as the step kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dpf_kernels.hpp"

namespace dpf {

// t = 0, state in copy 0 (the plain DPF's initial proposals are written
// there from the prior held in copy 1), flags and evidence cleared.
static __global__ void k_reset(int* tcur, unsigned char* cur, unsigned char* act, uint32_t* flags, double* loglik,
                        uint32_t* lflags, int* fcount, int F) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= F) return;
  tcur[f] = 0;
  fcount[f] = 0;
  cur[f] = 6;  // copy 0; identity cloud slots in both copies
  act[f] = 1;
  flags[f] = 0u;
  loglik[f] = 0.0;
  lflags[f] = 0u;
}

// Element e of an array of per-filter segments: find the filter by binary
// search over the offsets (the arrays are sized by the host).
__device__ __forceinline__ int filter_of(const long long* off, int F, long long e) {
  int lo = 0, hi = F - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= e)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Export (dir = 0) or import (dir = 1) one per-particle array whose filter
// blocks start at `off[f] * width` (width = elements per unit of off).
static __global__ void k_state_copy(float* ext, float* buf0, float* buf1, const unsigned char* cur,
                             const long long* off, int F, long long n_units, int width, int dir) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_units * width) return;
  const int f = filter_of(off, F, e / width);
  float* buf = (cur[f] & 1) ? buf1 : buf0;
  if (dir == 0)
    ext[e] = buf[e];
  else
    buf0[e] = ext[e];
}

// Export (dir = 0) or import (dir = 1) of a look-ahead cloud array ([N][width]
// per filter in units of off = inner offsets, width = DZ * M for z or M for
// lam per outer particle): export reads particle i's cloud from slot
// ind[copy][oo + i]; import writes slot order (the caller sets ind to the
// identity).
static __global__ void k_state_copy_cloud(float* ext, float* buf0, float* buf1, const int* ind0, const int* ind1,
                                   const unsigned char* cur,
                                   const long long* ioff, const int* ooff, const int* fM, int F, long long n_units,
                                   int width, int dir) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_units * width) return;
  if (dir == 1) {
    buf0[e] = ext[e];
    return;
  }
  const int f = filter_of(ioff, F, e / width);
  const long long per = (long long)fM[f] * width;  // elements per outer particle
  const long long loc = e - ioff[f] * width;
  const long long i = loc / per, rem = loc - i * per;
  const int c = cur[f] & 1;
  const int* ind = c ? ind1 : ind0;
  const bool ident = (cur[f] >> (1 + c)) & 1;
  const float* buf = c ? buf1 : buf0;
  ext[e] = buf[ioff[f] * width + (ident ? i : (long long)ind[ooff[f] + i]) * per + rem];
}

// x is [DX][NT]: element e = d * NT + g, filter by g.
static __global__ void k_state_copy_x(float* ext, float* buf0, float* buf1, const unsigned char* cur,
                               const long long* ooff64, int F, int NT, int DX, int dir) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)NT * DX) return;
  const int f = filter_of(ooff64, F, e % NT);
  float* buf = (cur[f] & 1) ? buf1 : buf0;
  if (dir == 0)
    ext[e] = buf[e];
  else
    buf0[e] = ext[e];
}

// Export of the time header: t[f] for f < F, zeros in the padding up to n_words.
static __global__ void k_export_time(const int* tcur, int* ext_t, int F, int n_words) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_words) return;
  ext_t[q] = q < F ? tcur[q] : 0;
}

static __global__ void k_import_time(const int* ext_t, int* tcur, unsigned char* cur, uint32_t* flags,
                              double* loglik, int F) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= F) return;
  tcur[f] = ext_t[f];
  cur[f] = 6;  // state in copy 0 in slot order
  flags[f] = 0u;
  loglik[f] = 0.0;
}

// ---------------------------------------------------------------- primitives
static __global__ void k_philox_words(Key key, const uint32_t* ctr, long long n, uint32_t* out) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const Words w = philox(key, ctr[4 * e], ctr[4 * e + 1], ctr[4 * e + 2], ctr[4 * e + 3]);
#pragma unroll
  for (int q = 0; q < 4; ++q) out[4 * e + q] = w.w[q];
}

template <int D>
static __global__ void k_normals_grid(Key key, uint32_t t, uint32_t purpose, int na, int nb, float* out) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)na * nb) return;
  const int a = (int)(e / nb), b = (int)(e % nb);
  float v[D];
  normals<D>(key, t, (uint32_t)a, (uint32_t)b, purpose, v);
#pragma unroll
  for (int d = 0; d < D; ++d) out[e * D + d] = v[d];
}

// Systematic resampling of one FP64 weight vector by the outer-resampling
// code of the step (group statistics, then points resolved 256 per
// workgroup by the same device function the new-cloud kernel uses).
static __global__ __launch_bounds__(kBlock) void k_prim_res_stats(const double* w, int n, double* gstat) {
  __shared__ ResScratch sh;
  float mg;
  double sg, qg;
  res_group_stat(LinSrc{w}, n, blockIdx.x, mg, sg, qg, sh);
  if (threadIdx.x == 0) {
    gstat[4 * blockIdx.x + 0] = (double)mg;
    gstat[4 * blockIdx.x + 1] = sg;
    gstat[4 * blockIdx.x + 2] = qg;
  }
}

static __global__ __launch_bounds__(kBlock) void k_prim_res_select(const double* w, int n, int n_out, double u,
                                                            const double* gstat, int* out) {
  __shared__ ResScratch sh;
  __shared__ int res[kBlock];
  const int G = (n + kResGroup - 1) / kResGroup;
  const int k0 = blockIdx.x * kBlock;
  const int np = min(kBlock, n_out - k0);
  resolve_points(LinSrc{w}, n, n_out, u, k0, np, gstat, G, res, sh, false);
  if (threadIdx.x < np) out[k0 + threadIdx.x] = res[threadIdx.x];
}

// One segment per (S index); the cdf build and search are those of k_newcloud.
template <int SEG, int JPT>
static __global__ __launch_bounds__(kBlock) void k_seg_systematic_prim(const double* w, int S, int n,
                                                                 int n_out, const double* u,
                                                                 int* out) {
  constexpr int NSEG = kBlock / SEG;
  __shared__ SegScratch sh;
  __shared__ double cdf[NSEG][SEG * JPT];
  const int s = threadIdx.x / SEG;
  const int ls = threadIdx.x % SEG;
  const int g = blockIdx.x * NSEG + s;
  const bool vg = g < S;
  double carry = 0.0;
#pragma unroll
  for (int r = 0; r < JPT; ++r) {
    const int j = ls + r * SEG;
    const double wj = (vg && j < n) ? w[(long long)g * n + j] : 0.0;
    double tot;
    const double c = seg_scan_incl<SEG>(wj, sh, tot);
    cdf[s][r * SEG + ls] = carry + c;
    carry += tot;
  }
  __syncthreads();
  if (!vg) return;
  const double uu = u[g];
  const double total = cdf[s][n - 1];
  for (int r = 0; r < JPT; ++r) {
    const int k = ls + r * SEG;
    if (k < n_out) out[(long long)g * n_out + k] = cdf_search(cdf[s], n, sys_point(k, uu, total, n_out));
  }
}

}  // namespace dpf
