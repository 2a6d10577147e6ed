// Counter-based random numbers on the device (gfx950).
//
// The paper does not say how random numbers are drawn; the library uses
// Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC'11), written here from that published
// definition.  A 4-word block is a pure function of
//   key     = (seed_lo32, seed_hi32 ^ filter_id)
//   counter = (t, a, b, purpose << 24 | block)
// so any particle can regenerate any of its draws without storing them.
//
// Transforms (exact in FP32 / FP64):
//   U24(w)      = (2 (w >> 9) + 1) 2^-24          in (0, 1)
//   U53(w0, w1) = ((w0 << 21) | (w1 >> 11)) 2^-53  in [0, 1)
//   R24(block)  = (2 v + 1) 2^-24                   in (0, 1),
//                 v = (w0 & 0x1ff) | (w1 & 0x1ff) << 9 | (w2 & 0x1f) << 18
// R24 is a block's remnant uniform, from 23 of the low bits U24 leaves
// unused.  Normals come from Box-Muller pairs on two uniforms (a, b):
// r = sqrt(-2 ln a), (r cos 2 pi b, r sin 2 pi b); within a block the slot
// pairs (w0, w1) and (w2, w3) give (U24, U24) pairs.  The FP32 transform
// uses the hardware log2 / sqrt / sin / cos (the sin and cos units take
// their argument in revolutions, so 2 pi b is never formed).
//
// Packed layout of a draw's normals, ten per two blocks: normal d = 10 q + r
// comes, for r < 8, from block 2q + r / 4 (slot pairs in order, cosine
// first), and for r = 8, 9 from the pair (R24(block 2q), R24(block 2q + 1)).
// A shorter draw is a prefix of a longer one.  The nested estimator's
// companion draws use the block-aligned layout (normal d from block d / 4),
// so that one block serves several companions (normals_k, normals_kb).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dpf {

enum Purpose : uint32_t {
  P_INIT_X = 0, P_INIT_Z = 1, P_LA_X = 2, P_LA_Z = 3, P_OUTER_U = 4, P_CAND_U = 5,
  P_INNER_U = 6, P_NEW_Z = 7, P_DPF_ANC_U = 8, P_DPF_X = 9, P_DPF_Z = 10,
  P_MDN_U = 11, P_MDN_X = 12, P_LA_B = 13
};

struct Key {
  uint32_t k0, k1;
};

__host__ __device__ inline Key make_key(uint64_t seed, uint32_t filter_id) {
  Key k;
  k.k0 = (uint32_t)seed;
  k.k1 = (uint32_t)(seed >> 32) ^ filter_id;
  return k;
}

struct Words {
  uint32_t w[4];
};

// Ten Philox4x32 rounds.  Each 32x32->64 product is one v_mad_u64_u32; each
// three-way exclusive or (hi(p) ^ c ^ k) one gfx950 v_bitop3_b32 (truth
// table 0x96, odd parity of its three inputs).
__device__ __forceinline__ Words philox(Key key, uint32_t c0, uint32_t c1, uint32_t c2,
                                        uint32_t c3) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t k0 = key.k0, k1 = key.k1;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t p0 = (uint64_t)M0 * c0;
    const uint64_t p1 = (uint64_t)M1 * c2;
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
    const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
  }
  Words o;
  o.w[0] = c0;
  o.w[1] = c1;
  o.w[2] = c2;
  o.w[3] = c3;
  return o;
}

__device__ __forceinline__ Words draw(Key key, uint32_t t, uint32_t a, uint32_t b,
                                      uint32_t purpose, uint32_t block) {
  return philox(key, t, a, b, (purpose << 24) | block);
}

// (2 floor(w / 2^9) + 1) / 2^24, the centre of one of 2^23 equal cells: the
// top 23 bits placed under the exponent of 1.0 (one v_alignbit_b32 forms
// 1 + floor(w / 2^9) 2^-23), minus 1 - 2^-24; the subtraction is exact (its
// operands lie within a factor of two of each other).
__device__ __forceinline__ float u24f(uint32_t w) {
  return __uint_as_float(__builtin_amdgcn_alignbit(0x7fu, w, 9u)) - 0x1.fffffep-1f;
}

__device__ __forceinline__ double u53(uint32_t w0, uint32_t w1) {
  const uint64_t v = ((uint64_t)w0 << 21) | (uint64_t)(w1 >> 11);
  return (double)v * 0x1p-53;
}

// The single U53 offset of a resampling / selection draw at counter (t, a, 0).
__device__ __forceinline__ double uniform53(Key key, uint32_t t, uint32_t a, uint32_t purpose) {
  const Words w = draw(key, t, a, 0u, purpose, 0u);
  return u53(w.w[0], w.w[1]);
}

// The U53 offset of a draw at counter (t, a, b).
__device__ __forceinline__ double uniform53_ab(Key key, uint32_t t, uint32_t a, uint32_t b, uint32_t purpose) {
  const Words w = draw(key, t, a, b, purpose, 0u);
  return u53(w.w[0], w.w[1]);
}

// The block's remnant uniform R24: the three fields joined under the
// exponent of 1.0 (1 + v 2^-23), minus 1 - 2^-24 (exact, as in u24f).
__device__ __forceinline__ float r24f(const Words& w) {
  const uint32_t v = (w.w[0] & 0x1ffu) | ((w.w[1] & 0x1ffu) << 9) | ((w.w[2] & 0x1fu) << 18);
  return __uint_as_float(0x3f800000u | v) - 0x1.fffffep-1f;
}

// Box-Muller pair in FP32 from two uniforms.
__device__ __forceinline__ void box_muller_u(float a, float b, float& n0, float& n1) {
  constexpr float kMinus2Ln2 = -1.3862943611198906f;  // -2 ln 2
  const float r = __builtin_amdgcn_sqrtf(kMinus2Ln2 * __builtin_amdgcn_logf(a));
  n0 = r * __builtin_amdgcn_cosf(b);
  n1 = r * __builtin_amdgcn_sinf(b);
}

// Box-Muller pair in FP32 from two words.
__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, float& n0, float& n1) {
  box_muller_u(u24f(wa), u24f(wb), n0, n1);
}

// D standard normals of the draw at counter (t, a, b) for one purpose
// (packed layout; blocks generated once, only those the D normals need).
template <int D>
__device__ __forceinline__ void normals(Key key, uint32_t t, uint32_t a, uint32_t b,
                                        uint32_t purpose, float* out) {
#pragma unroll
  for (int q = 0; q < (D + 9) / 10; ++q) {
    const int base = 10 * q;
    float rem[2] = {0.f, 0.f};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (base + 4 * h < D || base + 8 < D) {
        const Words w = draw(key, t, a, b, purpose, (uint32_t)(2 * q + h));
#pragma unroll
        for (int pr = 0; pr < 2; ++pr) {
          const int d0 = base + 4 * h + 2 * pr;
          if (d0 < D) {
            float n0, n1;
            box_muller(w.w[2 * pr], w.w[2 * pr + 1], n0, n1);
            out[d0] = n0;
            if (d0 + 1 < D) out[d0 + 1] = n1;
          }
        }
        if (base + 8 < D) rem[h] = r24f(w);
      }
    }
    if (base + 8 < D) {
      float n0, n1;
      box_muller_u(rem[0], rem[1], n0, n1);
      out[base + 8] = n0;
      if (base + 9 < D) out[base + 9] = n1;
    }
  }
}

// Normals D0 .. D1 - 1 of the draw at counter (t, a, b), packed layout,
// streamed in order as pairs: f(d, n_d, n_d+1) for even d.  Each block is
// generated once.  With kRem0 the caller has drawn block 0 itself (D0 >= 4,
// so none of its words are wanted here) and passes its remnant rem_b0.
template <int D0, int D1, bool kRem0, class F>
__device__ __forceinline__ void normal_pairs(Key key, uint32_t t, uint32_t a, uint32_t b, uint32_t purpose,
                                             float rem_b0, F&& f) {
  static_assert(D0 % 2 == 0 && D1 % 2 == 0 && D0 < D1, "normal_pairs: even, ordered bounds");
  static_assert(!kRem0 || (D0 >= 4 && D0 < 10), "normal_pairs: block 0 given, its words not wanted");
  float rem0 = rem_b0;
#pragma unroll
  for (int q = D0 / 10; q < (D1 + 9) / 10; ++q) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int lo = 10 * q + 4 * h;
      const bool want_words = lo + 4 > D0 && lo < D1;
      const bool want_rem = 10 * q + 8 >= D0 && 10 * q + 8 < D1;
      if (kRem0 && q == 0 && h == 0) continue;
      if (want_words || want_rem) {
        const Words w = draw(key, t, a, b, purpose, (uint32_t)(2 * q + h));
#pragma unroll
        for (int pr = 0; pr < 2; ++pr) {
          const int d = lo + 2 * pr;
          if (d >= D0 && d < D1) {
            float n0, n1;
            box_muller(w.w[2 * pr], w.w[2 * pr + 1], n0, n1);
            f(d, n0, n1);
          }
        }
        if (want_rem) {
          if (h == 0) {
            rem0 = r24f(w);
          } else {
            float n0, n1;
            box_muller_u(rem0, r24f(w), n0, n1);
            f(10 * q + 8, n0, n1);
          }
        }
      }
    }
  }
}

// Block-aligned layout (the nested estimator's companion draws): normals
// k D .. k D + D - 1 of the draw at counter (t, a, b), normal n from block
// n / 4, slot pairs as above.
template <int D>
__device__ __forceinline__ void normals_k(Key key, uint32_t t, uint32_t a, uint32_t b, uint32_t purpose, int k,
                                          float* out) {
  static_assert(D % 4 == 0 || D == 2 || D == 1, "normals_k: D must be 1, 2 or a multiple of 4");
  if constexpr (D % 4 == 0) {
    const uint32_t b0 = (uint32_t)k * (uint32_t)(D / 4);
#pragma unroll
    for (int blk = 0; blk < D / 4; ++blk) {
      const Words w = draw(key, t, a, b, purpose, b0 + (uint32_t)blk);
      box_muller(w.w[0], w.w[1], out[4 * blk], out[4 * blk + 1]);
      box_muller(w.w[2], w.w[3], out[4 * blk + 2], out[4 * blk + 3]);
    }
  } else if constexpr (D == 2) {
    const Words w = draw(key, t, a, b, purpose, (uint32_t)(k >> 1));
    const bool hi = (k & 1) != 0;
    box_muller(hi ? w.w[2] : w.w[0], hi ? w.w[3] : w.w[1], out[0], out[1]);
  } else {
    const Words w = draw(key, t, a, b, purpose, (uint32_t)(k >> 2));
    const bool hi = (k & 2) != 0;
    float n0, n1;
    box_muller(hi ? w.w[2] : w.w[0], hi ? w.w[3] : w.w[1], n0, n1);
    out[0] = (k & 1) ? n1 : n0;
  }
}

// Companions served by one Philox block of normals_k<D>: four for D = 1, two
// for D = 2, one (D / 4 blocks each) for D a multiple of 4.
template <int D>
constexpr int comp_per_block() {
  return D == 1 ? 4 : (D == 2 ? 2 : 1);
}

// normals_k<D> for k = k0 .. k0 + comp_per_block<D>() - 1 at once (k0 a
// multiple of that count), companion q's D normals at out[q D]: for D = 1
// and 2 the block's four normals in slot order, so one block serves them all.
template <int D>
__device__ __forceinline__ void normals_kb(Key key, uint32_t t, uint32_t a, uint32_t b, uint32_t purpose, int k0,
                                           float* out) {
  if constexpr (D == 1 || D == 2) {
    const Words w = draw(key, t, a, b, purpose, (uint32_t)(k0 / comp_per_block<D>()));
    box_muller(w.w[0], w.w[1], out[0], out[1]);
    box_muller(w.w[2], w.w[3], out[2], out[3]);
  } else {
    normals_k<D>(key, t, a, b, purpose, k0, out);
  }
}

}  // namespace dpf
