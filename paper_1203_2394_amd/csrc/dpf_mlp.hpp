// Learned proposal network: a mixture density network over x_t that stands
// in for the Monte Carlo optimal-proposal estimate of eq:approx3.
//
// Network: 32 (features, zero padded) -> 256 -> 256 -> 32 outputs (20 used:
// 4 mixture logits, 4 x 2 means, 4 x 2 log standard deviations), tanh-form
// GELU after both hidden layers.  Matrix products run on the gfx950 matrix
// cores, v_mfma_f32_16x16x32_bf16: BF16 operands (round to nearest even),
// FP32 accumulation.  Lane l of a wave holds, for a 16 x 16 x 32 step,
//   A: row l % 16, k = 8 (l / 16) .. 8 (l / 16) + 7   (8 bf16, 16 bytes)
//   B: col l % 16, the same 8 k                         (8 bf16, 16 bytes)
//   D: col l % 16, rows 4 (l / 16) .. 4 (l / 16) + 3    (4 floats)
// so both operands are read as 16-byte vectors from k-contiguous storage:
// weights as [out][in] (and transposed copies for the backward pass),
// activations row-major in LDS, batch-contiguous ("transposed") in HBM when
// the batch is the contraction index (weight gradients).
//
// Row tiles: a 256-thread workgroup (4 waves) owns 16 rows of the batch;
// wave w computes hidden columns 64 w .. 64 w + 63.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dpf_models.hpp"
#include "dpf_seg.hpp"

namespace dpf {

constexpr int kMlpIn = 32;
constexpr int kMlpHid = 256;
constexpr int kMlpOut = 32;
constexpr int kMix = 4;
constexpr int kMlpRows = 16;
constexpr float kLogSdMin = -6.907755278982137f;  // log 1e-3
constexpr float kLogSdMax = 6.907755278982137f;   // log 1e3

// Device blob of the network (bytes): BF16 weights [out][in], FP32 biases,
// and the feature standardisation (mean, standard deviation).
struct MlpBlobLayout {
  static constexpr size_t W1 = 0;                                  // bf16 [256][32]
  static constexpr size_t W2 = W1 + kMlpHid * kMlpIn * 2;          // bf16 [256][256]
  static constexpr size_t W3 = W2 + kMlpHid * kMlpHid * 2;         // bf16 [32][256]
  static constexpr size_t b1 = W3 + kMlpOut * kMlpHid * 2;         // f32 [256]
  static constexpr size_t b2 = b1 + kMlpHid * 4;                   // f32 [256]
  static constexpr size_t b3 = b2 + kMlpHid * 4;                   // f32 [32]
  static constexpr size_t fmean = b3 + kMlpOut * 4;                // f32 [32]
  static constexpr size_t fstd = fmean + kMlpIn * 4;               // f32 [32]
  static constexpr size_t bytes = fstd + kMlpIn * 4;
};

// FP32 parameter vector (training masters, Adam moments, gradients).
struct MlpParamLayout {
  static constexpr int W1 = 0;                          // [256][32]
  static constexpr int b1 = W1 + kMlpHid * kMlpIn;      // [256]
  static constexpr int W2 = b1 + kMlpHid;               // [256][256]
  static constexpr int b2 = W2 + kMlpHid * kMlpHid;     // [256]
  static constexpr int W3 = b2 + kMlpHid;               // [32][256]
  static constexpr int b3 = W3 + kMlpOut * kMlpHid;     // [32]
  static constexpr int n = b3 + kMlpOut;
};

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short bf16_t;

// Round to nearest even; NaN stays NaN.
__device__ __forceinline__ bf16_t f2bf(float v) {
  uint32_t u = __float_as_uint(v);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (bf16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ bf16x8 ld8(const bf16_t* p) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(p));
}

__device__ __forceinline__ f32x4 mfma16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

constexpr float kGeluC = 0.7978845608028654f;  // sqrt(2 / pi)
constexpr float kGeluA = 0.044715f;

__device__ __forceinline__ float gelu_f(float a) {
  const float th = tanh_f(kGeluC * (a + kGeluA * a * a * a));
  return 0.5f * a * (1.0f + th);
}
__device__ __forceinline__ float gelu_grad_f(float a) {
  const float th = tanh_f(kGeluC * (a + kGeluA * a * a * a));
  const float du = kGeluC * (1.0f + 3.0f * kGeluA * a * a);
  return 0.5f * (1.0f + th) + 0.5f * a * (1.0f - th * th) * du;
}

// LDS row strides (bf16 elements), padded by 16 bytes so that the 16 rows
// of an operand fragment fall on distinct banks.
constexpr int kInStride = kMlpIn + 8;
constexpr int kHidStride = kMlpHid + 8;

struct alignas(16) MlpShared {
  bf16_t x0[kMlpRows][kInStride];
  bf16_t h1[kMlpRows][kHidStride];
  bf16_t h2[kMlpRows][kHidStride];
  float part[2][kMlpRows][16];
  float o[kMlpRows][kMlpOut + 1];  // outputs of the tile (for an epilogue per row)
};

// Optional outputs of the training forward pass (batch B, row-major a1 / a2,
// batch-contiguous bf16 copies of the layer inputs).
struct MlpTrainOut {
  float* a1;   // [B][256] pre-activation of layer 1
  float* a2;   // [B][256]
  bf16_t* x0t;  // [32][B]
  bf16_t* h1t;  // [256][B]
  bf16_t* h2t;  // [256][B]
  int B;
};

// Weight fragments and biases of one wave, loaded before the layer inputs
// are ready so that the three layers find their operands in registers.
// Wave w owns hidden columns 64w..64w+63 (4 column tiles) and, in the output
// layer, column tile w & 1 over k-steps 4 (w >> 1) .. 4 (w >> 1) + 3.
struct MlpFrags {
  bf16x8 w1[1][4];
  bf16x8 w2[8][4];
  bf16x8 w3[4];
  float b1[4], b2[4], b3;
};

__device__ __forceinline__ void mlp_load_frags(const unsigned char* blob, MlpFrags& fr) {
  using BL = MlpBlobLayout;
  const bf16_t* W1 = reinterpret_cast<const bf16_t*>(blob + BL::W1);
  const bf16_t* W2 = reinterpret_cast<const bf16_t*>(blob + BL::W2);
  const bf16_t* W3 = reinterpret_cast<const bf16_t*>(blob + BL::W3);
  const float* b1 = reinterpret_cast<const float*>(blob + BL::b1);
  const float* b2 = reinterpret_cast<const float*>(blob + BL::b2);
  const float* b3 = reinterpret_cast<const float*>(blob + BL::b3);
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int lr = l & 15, lk = 8 * (l >> 4);
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const int n = 64 * w + 16 * nt + lr;
    fr.w1[0][nt] = ld8(W1 + (size_t)n * kMlpIn + lk);
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) fr.w2[ks][nt] = ld8(W2 + (size_t)n * kMlpHid + 32 * ks + lk);
    fr.b1[nt] = b1[n];
    fr.b2[nt] = b2[n];
  }
  const int n3 = 16 * (w & 1) + lr, k3 = 4 * (w >> 1);
#pragma unroll
  for (int q = 0; q < 4; ++q) fr.w3[q] = ld8(W3 + (size_t)n3 * kMlpHid + 32 * (k3 + q) + lk);
  fr.b3 = b3[n3];
}

// Hidden layer: rows of `in` (LDS, K = KIN) times the wave's weight
// fragments plus bias, GELU, rounded into `out` (LDS).
template <int KIN, int SIN, bool TRAIN>
__device__ __forceinline__ void mlp_hidden(const bf16_t (*in)[SIN], const bf16x8 (*wf)[4], const float* bias,
                                           bf16_t (*out)[kHidStride], int row0, float* a_out,
                                           bf16_t* h_t, int B) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int lr = l & 15, lk = 8 * (l >> 4);
  f32x4 acc[4];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ks = 0; ks < KIN / 32; ++ks) {
    const bf16x8 a = ld8(&in[lr][32 * ks + lk]);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = mfma16(a, wf[ks][nt], acc[nt]);
  }
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const int n = 64 * w + 16 * nt + lr;
    const float bn = bias[nt];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 4 * (l >> 4) + r;
      const float v = acc[nt][r] + bn;
      const bf16_t h = f2bf(gelu_f(v));
      out[row][n] = h;
      if constexpr (TRAIN) {
        const int g = row0 + row;
        if (g < B) {
          a_out[(size_t)g * kMlpHid + n] = v;
          h_t[(size_t)n * B + g] = h;
        }
      }
    }
  }
}

// The three layers for the 16 rows in sh.x0; outputs [rows][32] FP32.
template <bool TRAIN>
__device__ void mlp_rows(const MlpFrags& fr, MlpShared& sh, int row0, int nrows, float* out,
                         const MlpTrainOut& tr) {
  mlp_hidden<kMlpIn, kInStride, TRAIN>(sh.x0, fr.w1, fr.b1, sh.h1, row0, tr.a1, tr.h1t, tr.B);
  __syncthreads();
  mlp_hidden<kMlpHid, kHidStride, TRAIN>(sh.h1, fr.w2, fr.b2, sh.h2, row0, tr.a2, tr.h2t, tr.B);
  __syncthreads();
  // output layer: 2 column tiles x 8 k-steps, split over the 4 waves
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int lr = l & 15, lk = 8 * (l >> 4);
  const int nt = w & 1, kh = w >> 1;
  f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int q = 0; q < 4; ++q) acc = mfma16(ld8(&sh.h2[lr][32 * (4 * kh + q) + lk]), fr.w3[q], acc);
  if (kh == 1) {
#pragma unroll
    for (int r = 0; r < 4; ++r) sh.part[nt][4 * (l >> 4) + r][lr] = acc[r];
  }
  __syncthreads();
  if (kh == 0) {
    const int n = 16 * nt + lr;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 4 * (l >> 4) + r;
      const float v = (acc[r] + sh.part[nt][row][lr]) + fr.b3;
      sh.o[row][n] = v;
      if (row < nrows) out[(size_t)(row0 + row) * kMlpOut + n] = v;
    }
  }
}

// Standardised FP32 features X [B][32] -> outputs [B][32] (TRAIN: also the
// activations the backward pass needs).
template <bool TRAIN>
static __global__ __launch_bounds__(kBlock) void k_mlp_fwd_x(const unsigned char* blob, const float* X, int B,
                                                      float* out, MlpTrainOut tr) {
  __shared__ MlpShared sh;
  MlpFrags fr;
  mlp_load_frags(blob, fr);
  const int row0 = blockIdx.x * kMlpRows;
  const int nrows = min(kMlpRows, B - row0);
  for (int e = threadIdx.x; e < kMlpRows * kMlpIn; e += kBlock) {
    const int r = e / kMlpIn, c = e % kMlpIn;
    const bf16_t v = r < nrows ? f2bf(X[(size_t)(row0 + r) * kMlpIn + c]) : (bf16_t)0;
    sh.x0[r][c] = v;
    if (TRAIN && r < nrows) tr.x0t[(size_t)c * B + row0 + r] = v;
  }
  __syncthreads();
  mlp_rows<TRAIN>(fr, sh, row0, nrows, out, tr);
}

// ---------------------------------------------------------------- MDN
// Output row: logits [0, 4), means [4, 4 + 4 DX) as [component][d], log
// standard deviations [4 + 4 DX, 4 + 8 DX) likewise, clamped to
// [log 1e-3, log 1e3].
template <int DX>
struct Mdn {
  static constexpr int kMu = kMix, kSd = kMix + kMix * DX, kUsed = kMix + 2 * kMix * DX;
  static_assert(kUsed <= kMlpOut, "mixture does not fit the output layer");
};

__device__ __forceinline__ float clamp_sd(float s) { return fminf(fmaxf(s, kLogSdMin), kLogSdMax); }

// log q(x) of the mixture in row o.
template <int DX>
__device__ float mdn_logpdf(const float* o, const float* x) {
  using Q = Mdn<DX>;
  float lmax = -INFINITY;
#pragma unroll
  for (int c = 0; c < kMix; ++c) lmax = fmaxf(lmax, o[c]);
  float se = 0.f;
#pragma unroll
  for (int c = 0; c < kMix; ++c) se += fast_exp(o[c] - lmax);
  const float lse_l = lmax + fast_log(se);
  float e[kMix], emax = -INFINITY;
#pragma unroll
  for (int c = 0; c < kMix; ++c) {
    float q = 0.f;
#pragma unroll
    for (int d = 0; d < DX; ++d) {
      const float s = clamp_sd(o[Q::kSd + c * DX + d]);
      const float z = (x[d] - o[Q::kMu + c * DX + d]) * fast_exp(-s);
      q += -0.5f * z * z - s - 0.5f * kLn2Pi;
    }
    e[c] = (o[c] - lse_l) + q;
    emax = fmaxf(emax, e[c]);
  }
  float s2 = 0.f;
#pragma unroll
  for (int c = 0; c < kMix; ++c) s2 += fast_exp(e[c] - emax);
  return emax + fast_log(s2);
}

// Mean negative log-likelihood gradient: one row per thread.  Writes the
// gradient w.r.t. the outputs (divided by B) as bf16 row-major [B][32] and
// batch-contiguous [32][B], per-workgroup column sums (FP32, bias of the
// output layer) and the FP64 sum of the row NLLs.
template <int DX>
static __global__ __launch_bounds__(kBlock) void k_mdn_grad(const float* out, const float* xt, int B, bf16_t* gb,
                                                     bf16_t* gt, float* b3_part, double* loss_part) {
  using Q = Mdn<DX>;
  __shared__ float red[kBlock / kWave][kMlpOut];
  __shared__ double dred[kBlock / kWave];
  const int b = blockIdx.x * kBlock + threadIdx.x;
  const bool vb = b < B;
  float g[kMlpOut];
#pragma unroll
  for (int c = 0; c < kMlpOut; ++c) g[c] = 0.f;
  double nll = 0.0;
  if (vb) {
    float o[Q::kUsed], x[DX];
#pragma unroll
    for (int c = 0; c < Q::kUsed; ++c) o[c] = out[(size_t)b * kMlpOut + c];
#pragma unroll
    for (int d = 0; d < DX; ++d) x[d] = xt[(size_t)b * DX + d];
    float lmax = -INFINITY;
#pragma unroll
    for (int c = 0; c < kMix; ++c) lmax = fmaxf(lmax, o[c]);
    float se = 0.f;
#pragma unroll
    for (int c = 0; c < kMix; ++c) se += fast_exp(o[c] - lmax);
    const float lse_l = lmax + fast_log(se);
    float ell[kMix], emax = -INFINITY;
    float zz[kMix][DX], sd_inv[kMix][DX];
#pragma unroll
    for (int c = 0; c < kMix; ++c) {
      float q = 0.f;
#pragma unroll
      for (int d = 0; d < DX; ++d) {
        const float s = clamp_sd(o[Q::kSd + c * DX + d]);
        sd_inv[c][d] = fast_exp(-s);
        zz[c][d] = (x[d] - o[Q::kMu + c * DX + d]) * sd_inv[c][d];
        q += -0.5f * zz[c][d] * zz[c][d] - s - 0.5f * kLn2Pi;
      }
      ell[c] = (o[c] - lse_l) + q;
      emax = fmaxf(emax, ell[c]);
    }
    float s2 = 0.f;
#pragma unroll
    for (int c = 0; c < kMix; ++c) s2 += fast_exp(ell[c] - emax);
    const float L = emax + fast_log(s2);
    nll = -(double)L;
    const float invB = 1.0f / (float)B;
#pragma unroll
    for (int c = 0; c < kMix; ++c) {
      const float gam = fast_exp(ell[c] - L);
      const float pi = fast_exp(o[c] - lse_l);
      g[c] = (pi - gam) * invB;
#pragma unroll
      for (int d = 0; d < DX; ++d) {
        const float sr = o[Q::kSd + c * DX + d];
        const bool inside = sr > kLogSdMin && sr < kLogSdMax;
        g[Q::kMu + c * DX + d] = -gam * zz[c][d] * sd_inv[c][d] * invB;
        g[Q::kSd + c * DX + d] = inside ? -gam * (zz[c][d] * zz[c][d] - 1.0f) * invB : 0.f;
      }
    }
#pragma unroll
    for (int c = 0; c < kMlpOut; ++c) {
      const bf16_t h = f2bf(g[c]);
      gb[(size_t)b * kMlpOut + c] = h;
      gt[(size_t)c * B + b] = h;
    }
  }
  // column sums and the NLL sum, waves in order
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < kMlpOut; ++c) {
    const float v = seg_reduce_wave<OpAdd, kWave>(g[c]);
    if ((threadIdx.x & 63) == 0) red[w][c] = v;
  }
  const double nv = seg_reduce_wave<OpAdd, kWave>(nll);
  if ((threadIdx.x & 63) == 0) dred[w] = nv;
  __syncthreads();
  if (threadIdx.x < kMlpOut) {
    const int c = threadIdx.x;
    b3_part[(size_t)blockIdx.x * kMlpOut + c] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
  }
  if (threadIdx.x == 0) loss_part[blockIdx.x] = ((dred[0] + dred[1]) + dred[2]) + dred[3];
}

// ---------------------------------------------------------------- backward
// Per 16-row tile: dh2 = g W3, da2 = dh2 * gelu'(a2), dh1 = da2 W2,
// da1 = dh1 * gelu'(a1).  W3t [256][32] and W2t [256][256] are the
// transposed bf16 weights (k-contiguous for these products).  Writes da2,
// da1 batch-contiguous (bf16) and per-tile column sums (bias gradients).
struct MlpBwdArgs {
  const bf16_t* gb;   // [B][32]
  const float* a1;    // [B][256]
  const float* a2;    // [B][256]
  const bf16_t* W3t;  // [256][32]
  const bf16_t* W2t;  // [256][256]
  bf16_t* da2t;       // [256][B]
  bf16_t* da1t;       // [256][B]
  float* b2_part;     // [tiles][256]
  float* b1_part;     // [tiles][256]
  int B;
};

// d = (rows of `in`) x Wt^T for 256 output columns, then * gelu'(a); stores
// the bf16 result into `out` (LDS, optional), batch-contiguous global and
// column sums.
template <int KIN, int SIN>
__device__ __forceinline__ void mlp_back_layer(const bf16_t (*in)[SIN], const bf16_t* Wt, const float* a,
                                               bf16_t (*out)[kHidStride], bf16_t* dt, float* bpart,
                                               int row0, int nrows, int B) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int lr = l & 15, lk = 8 * (l >> 4);
  f32x4 acc[4];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ks = 0; ks < KIN / 32; ++ks) {
    const bf16x8 av = ld8(&in[lr][32 * ks + lk]);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int n = 64 * w + 16 * nt + lr;
      acc[nt] = mfma16(av, ld8(Wt + (size_t)n * KIN + 32 * ks + lk), acc[nt]);
    }
  }
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const int n = 64 * w + 16 * nt + lr;
    float cs = 0.f;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 4 * (l >> 4) + r;
      float v = 0.f;
      if (row < nrows) v = acc[nt][r] * gelu_grad_f(a[(size_t)(row0 + row) * kMlpHid + n]);
      cs += v;
      const bf16_t h = f2bf(v);
      if (out) out[row][n] = h;
      if (row < nrows) dt[(size_t)n * B + row0 + row] = h;
    }
    // the four row groups of the column: lanes lr, lr+16, lr+32, lr+48
    cs += __shfl_xor(cs, 16);
    cs += __shfl_xor(cs, 32);
    if (l < 16) bpart[n] = cs;
  }
}

static __global__ __launch_bounds__(kBlock) void k_mlp_bwd(MlpBwdArgs p) {
  __shared__ alignas(16) bf16_t g_sh[kMlpRows][kInStride];
  __shared__ alignas(16) bf16_t da2_sh[kMlpRows][kHidStride];
  const int row0 = blockIdx.x * kMlpRows;
  const int nrows = min(kMlpRows, p.B - row0);
  for (int e = threadIdx.x; e < kMlpRows * kMlpOut; e += kBlock) {
    const int r = e / kMlpOut, c = e % kMlpOut;
    g_sh[r][c] = r < nrows ? p.gb[(size_t)(row0 + r) * kMlpOut + c] : (bf16_t)0;
  }
  __syncthreads();
  mlp_back_layer<kMlpOut, kInStride>(g_sh, p.W3t, p.a2, da2_sh, p.da2t, p.b2_part + (size_t)blockIdx.x * kMlpHid,
                                     row0, nrows, p.B);
  __syncthreads();
  mlp_back_layer<kMlpHid, kHidStride>(da2_sh, p.W2t, p.a1, nullptr, p.da1t,
                                      p.b1_part + (size_t)blockIdx.x * kMlpHid, row0, nrows, p.B);
}

// ------------------------------------------------------- weight gradients
// dW[m][n] = sum_b At[m][b] Ht[n][b] over one chunk of the batch (split-K:
// chunk c of kWgChunk rows writes partial c).  One job = one 32 x 32 block
// of one of the three weight matrices; each wave computes one 16 x 16 tile.
constexpr int kWgChunk = 512;

struct WgJob {
  const bf16_t* At;  // [M][B]
  const bf16_t* Ht;  // [N][B]
  float* part;       // [chunks][M][N]
  int M, N;
};

struct WgArgs {
  WgJob job[3];
  int blocks[3];  // 32 x 32 blocks per job
  int B, chunks;
};

static __global__ __launch_bounds__(kBlock) void k_mlp_wgrad(WgArgs p) {
  int blk = blockIdx.x;
  const int chunk = blockIdx.y;
  int j = 0;
  while (j < 2 && blk >= p.blocks[j]) {
    blk -= p.blocks[j];
    ++j;
  }
  const WgJob& jb = p.job[j];
  const int nb = jb.N / 32;
  const int m0 = 32 * (blk / nb), n0 = 32 * (blk % nb);
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int lr = l & 15, lk = 8 * (l >> 4);
  const int tm = m0 + 16 * (w >> 1), tn = n0 + 16 * (w & 1);
  const int b0 = chunk * kWgChunk, b1 = min(p.B, b0 + kWgChunk);
  const bf16_t* ap = jb.At + (size_t)(tm + lr) * p.B + lk;
  const bf16_t* hp = jb.Ht + (size_t)(tn + lr) * p.B + lk;
  f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int b = b0; b < b1; b += 32) acc = mfma16(ld8(ap + b), ld8(hp + b), acc);
  float* out = jb.part + (size_t)chunk * jb.M * jb.N;
#pragma unroll
  for (int r = 0; r < 4; ++r) out[(size_t)(tm + 4 * (l >> 4) + r) * jb.N + tn + lr] = acc[r];
}

// ---------------------------------------------------------------- Adam
// One thread per parameter: gradient = ordered sum of the partials, Adam
// update of the FP32 master (moments m, v), BF16 / FP32 copies into the blob
// and the transposed BF16 copies used by the backward pass.
struct AdamArgs {
  float* p;  // masters [n]
  float* m;  // [n]
  float* v;  // [n]
  float* grad_out;  // [n] or null
  unsigned char* blob;
  bf16_t* W2t;  // [256][256]
  bf16_t* W3t;  // [256][32]
  const float* wpart[3];  // W1, W2, W3 partials [chunks][M][N]
  int chunks;
  const float* b1_part;   // [tiles][256]
  const float* b2_part;
  int tiles;
  const float* b3_part;   // [groups][32]
  int groups;
  const double* loss_part;
  float* loss;
  int B;
  float lr, bc1, bc2;  // bias corrections 1 - beta^t
  int update;          // 0: gradients only
};

constexpr float kAdamB1 = 0.9f, kAdamB2 = 0.999f, kAdamEps = 1e-8f;

// Writes parameter e of the FP32 vector into the blob (and the transposed copies).
__device__ __forceinline__ void mlp_store_param(int e, float val, unsigned char* blob, bf16_t* W2t, bf16_t* W3t) {
  using PL = MlpParamLayout;
  using BL = MlpBlobLayout;
  if (e < PL::b1) {
    reinterpret_cast<bf16_t*>(blob + BL::W1)[e] = f2bf(val);
  } else if (e < PL::W2) {
    reinterpret_cast<float*>(blob + BL::b1)[e - PL::b1] = val;
  } else if (e < PL::b2) {
    const int q = e - PL::W2;
    const bf16_t h = f2bf(val);
    reinterpret_cast<bf16_t*>(blob + BL::W2)[q] = h;
    if (W2t) W2t[(q % kMlpHid) * kMlpHid + q / kMlpHid] = h;
  } else if (e < PL::W3) {
    reinterpret_cast<float*>(blob + BL::b2)[e - PL::b2] = val;
  } else if (e < PL::b3) {
    const int q = e - PL::W3;
    const bf16_t h = f2bf(val);
    reinterpret_cast<bf16_t*>(blob + BL::W3)[q] = h;
    if (W3t) W3t[(q % kMlpHid) * kMlpOut + q / kMlpHid] = h;
  } else {
    reinterpret_cast<float*>(blob + BL::b3)[e - PL::b3] = val;
  }
}

static __global__ void k_mlp_adam(AdamArgs a) {
  using PL = MlpParamLayout;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e == 0 && a.loss) {
    double s = 0.0;
#pragma unroll 16
    for (int g = 0; g < a.groups; ++g) s += a.loss_part[g];
    *a.loss = (float)(s / a.B);
  }
  if (e >= PL::n) return;
  float g = 0.f;
  // (each sum unrolled: the loads of 16 partials in flight, added in order)
  if (e < PL::b1) {
#pragma unroll 16
    for (int c = 0; c < a.chunks; ++c) g += a.wpart[0][(size_t)c * (kMlpHid * kMlpIn) + e];
  } else if (e < PL::W2) {
#pragma unroll 16
    for (int t = 0; t < a.tiles; ++t) g += a.b1_part[(size_t)t * kMlpHid + e - PL::b1];
  } else if (e < PL::b2) {
#pragma unroll 16
    for (int c = 0; c < a.chunks; ++c) g += a.wpart[1][(size_t)c * (kMlpHid * kMlpHid) + e - PL::W2];
  } else if (e < PL::W3) {
#pragma unroll 16
    for (int t = 0; t < a.tiles; ++t) g += a.b2_part[(size_t)t * kMlpHid + e - PL::b2];
  } else if (e < PL::b3) {
#pragma unroll 16
    for (int c = 0; c < a.chunks; ++c) g += a.wpart[2][(size_t)c * (kMlpOut * kMlpHid) + e - PL::W3];
  } else {
#pragma unroll 16
    for (int t = 0; t < a.groups; ++t) g += a.b3_part[(size_t)t * kMlpOut + e - PL::b3];
  }
  if (a.grad_out) a.grad_out[e] = g;
  if (!a.update) return;
  const float m = kAdamB1 * a.m[e] + (1.0f - kAdamB1) * g;
  const float v = kAdamB2 * a.v[e] + (1.0f - kAdamB2) * g * g;
  a.m[e] = m;
  a.v[e] = v;
  const float mh = m / a.bc1, vh = v / a.bc2;
  const float p = a.p[e] - a.lr * mh / (sqrtf(vh) + kAdamEps);
  a.p[e] = p;
  mlp_store_param(e, p, a.blob, a.W2t, a.W3t);
}

// Masters -> blob (and transposed copies when W2t / W3t are given), plus the
// feature standardisation.
static __global__ void k_mlp_pack(const float* params, const float* fmean, const float* fstd, unsigned char* blob,
                           bf16_t* W2t, bf16_t* W3t) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < MlpParamLayout::n) mlp_store_param(e, params[e], blob, W2t, W3t);
  if (e < kMlpIn) {
    reinterpret_cast<float*>(blob + MlpBlobLayout::fmean)[e] = fmean[e];
    reinterpret_cast<float*>(blob + MlpBlobLayout::fstd)[e] = fstd[e];
  }
}

}  // namespace dpf
