// dpf_data.hip: preparing the learned proposal's training set on the device
// -- feature statistics, standardisation, the per-epoch shuffle and the
// gather of a batch -- so that the training loop only sequences calls.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "dpf_engine.hpp"

namespace dpf {

namespace {

constexpr int kStatThreads = 256;
constexpr int kStatCols = 32;                          // columns handled at once
constexpr int kStatRowLanes = kStatThreads / kStatCols;  // rows in flight per column

// Mean and sample standard deviation of each column of X [n][ld] (first
// `cols` columns): one workgroup; thread t takes column t % 32 and the rows
// r = t / 32 (mod 8); FP64 sums, combined in a fixed order, two passes
// (mean, then centred squares).
__global__ __launch_bounds__(kStatThreads) void k_feature_stats(const float* X, long long n, int cols, int ld,
                                                                float* mean, float* sdev, float floor_sd) {
  __shared__ double part[kStatRowLanes][kStatCols];
  __shared__ double mu[kStatCols];
  const int c = threadIdx.x % kStatCols, r0 = threadIdx.x / kStatCols;
  for (int c0 = 0; c0 < cols; c0 += kStatCols) {
    const int col = c0 + c;
    const bool on = col < cols;
    double s = 0.0;
    if (on)
      for (long long r = r0; r < n; r += kStatRowLanes) s += (double)X[r * ld + col];
    part[r0][c] = s;
    __syncthreads();
    if (r0 == 0) {
      double t = 0.0;
      for (int q = 0; q < kStatRowLanes; ++q) t += part[q][c];
      mu[c] = t / (double)n;
    }
    __syncthreads();
    const double m = mu[c];
    double v = 0.0;
    if (on)
      for (long long r = r0; r < n; r += kStatRowLanes) {
        const double d = (double)X[r * ld + col] - m;
        v += d * d;
      }
    part[r0][c] = v;
    __syncthreads();
    if (r0 == 0 && on) {
      double t = 0.0;
      for (int q = 0; q < kStatRowLanes; ++q) t += part[q][c];
      mean[col] = (float)m;
      sdev[col] = fmaxf((float)sqrt(t / (double)(n - 1)), floor_sd);
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBlock) void k_standardize(const float* X, long long n, int cols, int ld,
                                                       const float* mean, const float* sdev, float* out,
                                                       int ld_out) {
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n * ld_out) return;
  const long long r = e / ld_out;
  const int c = (int)(e - r * ld_out);
  out[e] = c < cols ? (X[r * ld + c] - mean[c]) / sdev[c] : 0.0f;
}

// A keyed bijection of [0, 2^(2h)): four Feistel rounds on two h-bit
// halves, each round function the low h bits of a Philox4x32-10 word keyed
// by (seed, round) over (half, epoch).  A Feistel network is a permutation
// for any round function; with a pseudo-random one, four rounds give a
// pseudo-random permutation (Luby and Rackoff).
__device__ __forceinline__ uint32_t feistel(Key key, uint32_t epoch, uint32_t x, int h) {
  const uint32_t mask = (1u << h) - 1u;
  uint32_t L = x >> h, R = x & mask;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const Words w = philox(key, R, epoch, (uint32_t)q, 0xA5u);
    const uint32_t nl = R;
    R = L ^ (w.w[0] & mask);
    L = nl;
  }
  return (L << h) | R;
}

// perm[i]: the bijection applied to i, then again while the value lies at
// or beyond n (cycle walking): the first value below n on i's cycle, which
// exists because i itself is below n.  A permutation of [0, n).
__global__ __launch_bounds__(kBlock) void k_permutation(Key key, uint32_t epoch, long long n, int h, int* perm) {
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  uint32_t y = feistel(key, epoch, (uint32_t)i, h);
  while ((long long)y >= n) y = feistel(key, epoch, y, h);
  perm[i] = (int)y;
}

__global__ __launch_bounds__(kBlock) void k_gather_rows(const float* src, long long n_src, int cols, int ld_src,
                                                       const int* idx, int count, float* dst, int ld_dst) {
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (e >= (long long)count * cols) return;
  const int k = (int)(e / cols), c = (int)(e - (long long)k * cols);
  const int r = idx[k];
  dst[(long long)k * ld_dst + c] = (r >= 0 && r < n_src) ? src[(long long)r * ld_src + c] : NAN;
}

}  // namespace

}  // namespace dpf

using namespace dpf;

extern "C" dpf_status dpf_feature_stats(const float* d_X, int64_t n, int32_t cols, int32_t ld, float* d_mean,
                                        float* d_std, float std_floor, void* hip_stream) {
  if (!d_X || !d_mean || !d_std) return fail(DPF_EINVAL, "null buffer");
  if (n < 2 || cols < 1 || ld < cols) return fail(DPF_EINVAL, "need n >= 2 rows and 1 <= cols <= ld (n=%lld cols=%d ld=%d)",
                                                  (long long)n, cols, ld);
  if (!(std_floor >= 0.0f)) return fail(DPF_EINVAL, "std_floor must be >= 0");
  hipLaunchKernelGGL(k_feature_stats, dim3(1), dim3(kStatThreads), 0, (hipStream_t)hip_stream, d_X, (long long)n,
                     cols, ld, d_mean, d_std, std_floor);
  LAUNCH_CHECK("k_feature_stats");
  return DPF_OK;
}

extern "C" dpf_status dpf_standardize(const float* d_X, int64_t n, int32_t cols, int32_t ld, const float* d_mean,
                                      const float* d_std, float* d_out, int32_t ld_out, void* hip_stream) {
  if (n < 0 || cols < 0 || ld < cols || ld_out < cols) return fail(DPF_EINVAL, "bad sizes");
  if (n == 0 || ld_out == 0) return DPF_OK;
  if (!d_X || !d_mean || !d_std || !d_out) return fail(DPF_EINVAL, "null buffer");
  const long long tot = (long long)n * ld_out;
  if ((tot + kBlock - 1) / kBlock > 0x7fffffffLL) return fail(DPF_EINVAL, "too many elements");
  hipLaunchKernelGGL(k_standardize, dim3((unsigned)((tot + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     (hipStream_t)hip_stream, d_X, (long long)n, cols, ld, d_mean, d_std, d_out, ld_out);
  LAUNCH_CHECK("k_standardize");
  return DPF_OK;
}

extern "C" dpf_status dpf_permutation(uint64_t seed, uint32_t epoch, int64_t n, int32_t* d_perm, void* hip_stream) {
  if (n < 0 || n > 0x7fffffffLL) return fail(DPF_EINVAL, "n = %lld outside 0..2^31-1", (long long)n);
  if (n == 0) return DPF_OK;
  if (!d_perm) return fail(DPF_EINVAL, "null buffer");
  int h = 1;  // halves of h bits: 2^(2h) >= n
  while ((1LL << (2 * h)) < n) ++h;
  hipLaunchKernelGGL(k_permutation, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     (hipStream_t)hip_stream, make_key(seed, 0xDA7Au), epoch, (long long)n, h, d_perm);
  LAUNCH_CHECK("k_permutation");
  return DPF_OK;
}

extern "C" dpf_status dpf_gather_rows(const float* d_src, int64_t n_src, int32_t cols, int32_t ld_src,
                                      const int32_t* d_idx, int32_t count, float* d_dst, int32_t ld_dst,
                                      void* hip_stream) {
  if (n_src < 0 || cols < 0 || ld_src < cols || ld_dst < cols || count < 0) return fail(DPF_EINVAL, "bad sizes");
  if (count == 0 || cols == 0) return DPF_OK;
  if (!d_src || !d_idx || !d_dst) return fail(DPF_EINVAL, "null buffer");
  const long long tot = (long long)count * cols;
  hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((tot + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     (hipStream_t)hip_stream, d_src, (long long)n_src, cols, ld_src, d_idx, count, d_dst, ld_dst);
  LAUNCH_CHECK("k_gather_rows");
  return DPF_OK;
}
