// Step kernels of the look-ahead DPF (Section 2.2, Fig. 4) and of the plain
// DPF (Section 2, Fig. 2) for many independent filters of uneven sizes.
//
// Data layout in HBM (filter f, outer offset oo = ooff[f], inner offset
// io = ioff[f], sizes N = fN[f], M = fM[f]):
//   x    [DX][NT]            x[d * NT + oo + i]          (SoA, coalesced over i)
//   z    [sum N*DZ*M]         z[(io + i*M) * DZ + d*M + j] ([N][DZ][M] per filter)
//   lam  [sum N*M]            lam[io + i*M + j]           (log qbar, eq:qbar)
//   ell  [sum N*M]            look-ahead / measurement log-weights
//   logw [NT], anc [NT], sel [NT], kpart [NT][DZ]
// x, z and lam are double-buffered; cur[f] says which copy holds the state of
// filter f, so filters that sit a step out keep their state without a copy.
//
// A step is four launches: weights (one workgroup per tile of outer
// particles), two small resampling kernels (one workgroup per group of 256
// outer weights), and the new-cloud kernel, whose last workgroup per filter
// also forms the estimates and advances the filter (no separate launch).
//
// Per-particle kernels run one 256-thread workgroup per tile of 256/SEG
// consecutive outer particles of one filter (a "segment" of SEG lanes per
// particle, lane l handling inner indices l, l+SEG, ..., up to SEG*JPT).
#pragma once
#include <hip/hip_runtime.h>
#include <limits.h>
#include <math.h>
#include <stdint.h>

#include "dpf_models.hpp"
#include "dpf_proj.hpp"
#include "dpf_rng.hpp"
#include "dpf_seg.hpp"

namespace dpf {

enum FlagBits : uint32_t {
  F_DEGENERATE_OUTER = 1u,
  F_DEGENERATE_INNER = 2u,
  F_NONFINITE = 4u,
  F_FALLBACK = 8u
};

constexpr int kResGroup = 256;  // outer weights per resampling workgroup
constexpr int kFeatMax = 32;    // input width of the learned-proposal network

// Models whose outer-particle features [x, y, cloud mean, cloud variance] fit
// the network keep the per-particle cloud moments up to date when asked.
template <class Mdl>
constexpr bool has_moments() { return Mdl::DX + Mdl::DY + 2 * Mdl::DZ <= kFeatMax; }

// Models whose predicted observation the look-ahead pass can form (they
// provide obs_mean).
template <class Mdl>
constexpr bool has_yhat() { return Mdl::DY == 1; }

// Number of z-free terms of log p(x' | x, z) (px_pre); 1 for models whose
// transition of x ignores z (unused there).
template <class Mdl>
constexpr int npx() {
  if constexpr (Mdl::kXdepZ) return Mdl::NPX;
  else return 1;
}

// Per-filter bookkeeping for the resampling groups.
struct FilterInfo {
  int rg_base;  // first resampling group of the filter
  int ngroup;   // its number of groups
  int pad0, pad1;
};

struct StepArgs {
  const float* prm;
  const int4* tiles;  // (filter, first outer index, tile index within filter, first resampling group)
  const int* fN;
  const int* fM;
  const int* ooff;
  const long long* ioff;
  const FilterInfo* finfo;
  int NT;
  int advance;   // 1: a step (time advances, estimates); 0: initialisation
  uint64_t seed;
  int* tcur;             // [F] time of the state (advanced by the statistics kernel)
  unsigned char* cur;    // [F] bit 0: copy holding the state (flipped with the time);
                         // bits 1, 2: copy 0 / copy 1 has identity cloud slots
  unsigned char* act;    // [F] whether the filter takes the current step (set by the weights kernel)
  const unsigned char* active;  // [F] or null
  const int* run_Tf;            // [F] or null: filter steps while tcur < min(run_Tf, run_T)
  int run_T;
  const float* Y;
  long long y_tstride;  // y of filter f at time t: Y + (t-1) * y_tstride + f * DY
  float* x[2];
  float* z[2];
  float* lam[2];
  float* ell;
  float* logw;
  int* anc;
  int* sel;      // [NT] selected candidate (look-ahead) / inner ancestor (plain)
  float* kpart;  // [NT][DZ] per-particle sum_j qbar z (plain: of the proposals)
  double* gstat;  // [resampling groups + 64][4]: group max log w, sum, sum of squares (group scale)
  double* fstat;  // [F][4]: max log w, sum w, sum w^2, degenerate (0/1)
  float* ess;     // [F]
  double* dlogz;  // [F]
  double* loglik;  // [F] cumulative
  uint32_t* flags;  // [F]
  float* est_x;     // [F][DX]
  float* est_z;     // [F][DZ]
  float* trace_x;   // [T][F][DX] or null
  float* trace_z;   // [T][F][DZ] or null
  int n_filters;
  int dy;
  int dx, dz;
  int n_tiles;  // tiles of the class being launched (tile-looping kernels)
  int anc_ready;  // outer ancestors already in anc
  const int2* rgroups;  // (filter, group) of each resampling workgroup
  const int4* ginfo;    // per resampling group: its filter's (first outer index, N, first group, groups)
  int n_commit;         // learned-step commit workgroups at the head of the launch
  int n_comp;           // companions per look-ahead candidate (nested estimator; 0: paired)
  // predicted observation (models with a one-dimensional y), or null: per
  // outer particle sum_j qbar h(xla, zla) of this step's look-ahead draws
  // (yp) and of the next step's (yp_next, written by a fused new-cloud
  // launch); the filter's yhat and its trace
  float* yp;
  float* yp_next;
  float* est_y;    // [F]
  float* trace_y;  // [T][F] or null
  // look-ahead state: cloud slot of each outer particle, per copy.  A step
  // that resamples by copying writes the identity; the learned step writes
  // its outer ancestors instead of moving the clouds.
  int* ind[2];
  float* mom;  // [NT][2 DZ] qbar-weighted cloud mean and variance, or null (not maintained)
  // learned step
  const unsigned char* mlp;  // network blob
  float* mdn;                // [NT][32] network outputs for the current step
  float* xtmp;               // [DX][NT] proposals x_t before resampling
  float* logq;               // [NT] log q of the proposals
  float* kpart_tmp;          // [NT][DZ]
  float* mom_tmp;            // [NT][2 DZ]
  unsigned char* fb;         // [F] 1 where the look-ahead step replaces the learned one; null otherwise
  uint32_t* lflags;          // [F] flags of the learned pass, kept only if it is accepted
  double ess_frac;           // fallback threshold on ESS / N
  // look-ahead run: the new-cloud kernel also computes the next step's
  // look-ahead weights from the clouds it builds (null: it does not), and the
  // estimates kernel records which filters take the next step
  float* ell_next;
  float* logw_next;
  double* gpart;  // [resampling groups][DX + DZ] partial sums of the estimates
  int* fcount;    // [F] workgroups of the step-end kernel done (back to 0 by the last)
};

__device__ __forceinline__ int copy_of(unsigned char c) { return c & 1; }

// Every per-filter value a tile reads, fetched together: the empty asm needs
// them all before the early exits, so the loads go out in one round instead
// of a chain of dependent ones behind each branch.
struct FilterView {
  long long io;
  int N, M, oo, t, ngroup;
  int act, fb, cur;
};

__device__ __forceinline__ FilterView load_filter(const StepArgs& a, int f) {
  FilterView v;
  v.act = a.act[f];
  v.fb = a.fb != nullptr ? a.fb[f] : 1;
  v.N = a.fN[f];
  v.M = a.fM[f];
  v.oo = a.ooff[f];
  v.io = a.ioff[f];
  v.t = a.tcur[f];
  v.cur = a.cur[f];
  v.ngroup = a.finfo[f].ngroup;
  asm volatile("" ::"v"(v.act), "v"(v.fb), "v"(v.N), "v"(v.M), "v"(v.oo), "v"(v.io), "v"(v.t), "v"(v.cur),
               "v"(v.ngroup));
  return v;
}
__device__ __forceinline__ bool ident_slots(unsigned char c, int copy) { return (c >> (1 + copy)) & 1; }

// fz_pre (transition out of time ts) for a whole segment whose lanes share
// the outer particle: lane q of each wave's part of the segment evaluates
// component q once, and the components are broadcast (readlane within a
// wave, lane permutes when two segments share a wave) instead of every lane
// evaluating all of them.
template <class Mdl, int SEG>
__device__ __forceinline__ void fz_pre_seg(Prm P, const float* xp, const float* xn, int ts, float* pre) {
  constexpr int DZ = Mdl::DZ;
  constexpr int W = SEG < 64 ? SEG : 64;
  if constexpr (DZ > W || Mdl::NPRE != DZ) {
    Mdl::fz_pre(P, xp, xn, ts, pre);
  } else {
    const int lane = threadIdx.x & 63;
    const int q = lane % W;
    const float mine = Mdl::fz_pre_k(P, xp, xn, ts, q < DZ ? q : 0);
    if constexpr (W == 64) {
#pragma unroll
      for (int k = 0; k < DZ; ++k) pre[k] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(mine), k));
    } else {
      const int base = lane - q;
#pragma unroll
      for (int k = 0; k < DZ; ++k) pre[k] = __shfl(mine, base + k);
    }
  }
}

// Minimum waves per SIMD the compiler must leave room for: two for the
// wide-z models (their per-particle arrays would otherwise take the whole
// register file for one wave), no constraint otherwise.
template <class Mdl>
constexpr int min_waves() {
  return Mdl::kStreamZ ? 2 : 1;
}

// Whether filter f takes this step: the caller's mask and the run limits,
// evaluated by the weights kernel (before the time advances) and recorded in
// act[f] for the later kernels of the step.
__device__ __forceinline__ bool step_active(const StepArgs& a, int f) {
  if (a.active != nullptr && a.active[f] == 0) return false;
  const int lim = a.run_Tf ? min(a.run_Tf[f], a.run_T) : a.run_T;
  return a.tcur[f] < lim;
}

template <class Mdl>
__device__ __forceinline__ void load_y(const StepArgs& a, int f, int t, float* y) {
  const float* yp = a.Y + (long long)(t - 1) * a.y_tstride + (long long)f * Mdl::DY;
#pragma unroll
  for (int k = 0; k < Mdl::DY; ++k) y[k] = yp[k];
}

template <class Mdl>
__device__ __forceinline__ const float* y_row(const StepArgs& a, int f, int t) {
  return a.Y + (long long)(t - 1) * a.y_tstride + (long long)f * Mdl::DY;
}

// Online log-sum-exp accumulator (non-finite values are skipped).
struct Lse {
  float m = -INFINITY, s = 0.f;
  __device__ void add(float v) {
    if (!finitef(v)) return;
    if (v > m) {
      s = s * fast_exp(m - v) + 1.0f;
      m = v;
    } else {
      s += fast_exp(v - m);
    }
  }
};

template <int SEG>
__device__ __forceinline__ float seg_lse(Lse l, SegScratch& sh) {
  const float m = seg_max<SEG>(l.m, sh);
  const float sc = (l.m == -INFINITY) ? 0.f : l.s * fast_exp(l.m - m);
  const float s = seg_sum<SEG>(sc, sh);
  return (m == -INFINITY) ? -INFINITY : m + fast_log(s);
}

// Block-wide (256 threads) FP64 reductions and scans in a fixed order:
// DPP within each wave, then the four wave results in order.
__device__ __forceinline__ double block_sum_256(double v, double* red4) {
  v = seg_reduce_wave<OpAdd, kWave>(v);
  if ((threadIdx.x & (kWave - 1)) == 0) red4[threadIdx.x / kWave] = v;
  __syncthreads();
  const double r = ((red4[0] + red4[1]) + red4[2]) + red4[3];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double block_scan_incl_256(double v, double* red4) {
  const int w = threadIdx.x / kWave;
  v = seg_scan_wave<kWave>(v);
  if ((threadIdx.x & (kWave - 1)) == kWave - 1) red4[w] = v;
  __syncthreads();
  double pre = 0.0;
  for (int q = 0; q < w; ++q) pre += red4[q];
  __syncthreads();
  return v + pre;
}

// Block-wide stream compaction in thread order: the values of threads with
// pred go to out[0..total); returns total; incl receives the number of pred
// threads up to and including this one.
__device__ __forceinline__ int block_compact(bool pred, int value, int* out, int* wcnt, int* incl) {
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const unsigned long long b = __ballot(pred);
  const int r = __popcll(b & ((1ull << lane) - 1ull));
  if (lane == 0) wcnt[w] = __popcll(b);
  __syncthreads();
  int off = 0, total = 0;
#pragma unroll
  for (int q = 0; q < kBlock / kWave; ++q) {
    const int c = wcnt[q];
    if (q < w) off += c;
    total += c;
  }
  if (pred) out[off + r] = value;
  if (incl) *incl = off + r + (pred ? 1 : 0);
  __syncthreads();
  return total;
}

// ------------------------------------------------------------ initialisation
// Prior draws [x_0; z_0] ~ N(0, I) (INIT_X at (0, i, 0), INIT_Z at (0, i, j)).
// Look-ahead state: lam_0 = -log M, written to copy 0.  Plain DPF: the prior
// goes to copy 1 with ell = 0 and anc = identity, after which the proposal
// kernel runs with t = 0 (no y_0 is consumed).
template <class Mdl, int SEG, int JPT, bool PLAIN>
static __global__ __launch_bounds__(kBlock) void k_init(StepArgs a) {
  const int4 tile = a.tiles[blockIdx.x];
  const int f = tile.x;
  const int N = a.fN[f], M = a.fM[f];
  const int i = tile.y + threadIdx.x / SEG;
  const int ls = threadIdx.x % SEG;
  if (i >= N) return;
  const int oo = a.ooff[f];
  const long long io = a.ioff[f];
  const Key key = make_key(a.seed, (uint32_t)f);
  const int dst = PLAIN ? 1 : 0;
  if (ls == 0) {
    float x0[Mdl::DX];
    normals<Mdl::DX>(key, 0u, (uint32_t)i, 0u, P_INIT_X, x0);
#pragma unroll
    for (int d = 0; d < Mdl::DX; ++d) a.x[dst][(long long)d * a.NT + oo + i] = x0[d];
    if (PLAIN) a.anc[oo + i] = i;
  }
  const float lam0 = -fast_log((float)M);
  float* zrow = a.z[dst] + (io + (long long)i * M) * Mdl::DZ;
  for (int r = 0; r < JPT; ++r) {
    const int j = ls + r * SEG;
    if (j >= M) break;
    float z0[Mdl::DZ];
    normals<Mdl::DZ>(key, 0u, (uint32_t)i, (uint32_t)j, P_INIT_Z, z0);
#pragma unroll
    for (int d = 0; d < Mdl::DZ; ++d) zrow[d * M + j] = z0[d];
    if (PLAIN)
      a.ell[io + (long long)i * M + j] = 0.f;
    else
      a.lam[dst][io + (long long)i * M + j] = lam0;
  }
}

// ------------------------------------------------------- look-ahead weights
// Fig. 4 steps 1-2: for every (i, j) one candidate x from the j-th inner
// component (LA_X normals at (t, i, j)) and its companion z (LA_Z), then
// ell = lam + log p(y_t | xla, zla) (eq:weightsMC) and the per-particle
// log-sum-exp log w_i.

// log p(y_t | xla, zla) of inner particle (i, j) at time t from its outer x
// and its z; ell = lam + that (la_ell).
//
// The inputs pass through empty asm first: the compiler cannot merge this
// arithmetic with the caller's on the same values, so the weights kernel and
// the new-cloud kernel (a look-ahead run) compile it alike and get the same
// bits.
template <class Mdl, bool H = false>
__device__ __forceinline__ float la_logpy(const StepArgs& a, const Key& key, int t, int i, int j, const float* xi,
                                          const float* zi, const float* yi, float* hout = nullptr) {
  float x[Mdl::DX], z[Mdl::DZ], y[Mdl::DY];
#pragma unroll
  for (int d = 0; d < Mdl::DX; ++d) {
    x[d] = xi[d];
    asm volatile("" : "+v"(x[d]));
  }
#pragma unroll
  for (int d = 0; d < Mdl::DZ; ++d) {
    z[d] = zi[d];
    asm volatile("" : "+v"(z[d]));
  }
#pragma unroll
  for (int d = 0; d < Mdl::DY; ++d) y[d] = yi[d];
  // one draw per candidate: x's normals first, then z's
  float nu[Mdl::DX + Mdl::DZ], xl[Mdl::DX], pre[Mdl::NPRE], zl[Mdl::DZ], r0[Mdl::DY];
  normals<Mdl::DX + Mdl::DZ>(key, (uint32_t)t, (uint32_t)i, (uint32_t)j, P_LA_X, nu);
  Mdl::fx(as_prm(a.prm), x, z, nu, t - 1, xl);
  Mdl::fz_pre(as_prm(a.prm), x, xl, t - 1, pre);
  Mdl::fz_post(as_prm(a.prm), pre, z, nu + Mdl::DX, zl);
  Mdl::obs_pre(as_prm(a.prm), y, xl, r0);
  if constexpr (H) {
    // the noise-free observation of the draw, on opaque copies (no sharing
    // with the likelihood's arithmetic)
    float xh[Mdl::DX], zh[Mdl::DZ];
#pragma unroll
    for (int d = 0; d < Mdl::DX; ++d) {
      xh[d] = xl[d];
      asm volatile("" : "+v"(xh[d]));
    }
#pragma unroll
    for (int d = 0; d < Mdl::DZ; ++d) {
      zh[d] = zl[d];
      asm volatile("" : "+v"(zh[d]));
    }
    Mdl::obs_mean(as_prm(a.prm), xh, zh, hout);
  }
  return Mdl::logpy_post(as_prm(a.prm), r0, zl);
}

// The same for a wide-z model, for the 64 inner particles of a wave at once
// (converged code; lane l's particle j): the candidate's z component by
// component, each pair of components into the matrix-core residual
// (WaveProj; ca its A values, yrow the observation y_t).
template <class Mdl>
__device__ __forceinline__ float la_logpy_wave(const StepArgs& a, const Key& key, int t, int i, int j,
                                               const float* xi, const float* zi, const float* yrow,
                                               const float* ca) {
  static_assert(Mdl::kStreamZ && Mdl::DZ % 2 == 0 && Mdl::DX == 4,
                "la_logpy_wave: wide-z models, DX = 4, DZ even");
  const Prm P = as_prm(a.prm);
  float x[Mdl::DX], z[Mdl::DZ];
#pragma unroll
  for (int d = 0; d < Mdl::DX; ++d) {
    x[d] = xi[d];
    asm volatile("" : "+v"(x[d]));
  }
#pragma unroll
  for (int d = 0; d < Mdl::DZ; ++d) {
    z[d] = zi[d];
    asm volatile("" : "+v"(z[d]));
  }
  // the candidate's draw: block 0 gives x's four normals (and its remnant
  // uniform), z's normals 4 .. 4 + DZ - 1 follow in pairs
  float nu_x[Mdl::DX], xl[Mdl::DX], c[Mdl::NPL];
  const Words w0 = draw(key, (uint32_t)t, (uint32_t)i, (uint32_t)j, P_LA_X, 0u);
  box_muller(w0.w[0], w0.w[1], nu_x[0], nu_x[1]);
  box_muller(w0.w[2], w0.w[3], nu_x[2], nu_x[3]);
  Mdl::fx(P, x, z, nu_x, t - 1, xl);
  Mdl::fz_lite(P, x, xl, t - 1, c);
  WaveProj<Mdl> pj;
  pj.start();
  normal_pairs<Mdl::DX, Mdl::DX + Mdl::DZ, true>(
      key, (uint32_t)t, (uint32_t)i, (uint32_t)j, P_LA_X, r24f(w0), [&](int d, float n0, float n1) {
        const int kk = d - Mdl::DX;
        const float z0 = Mdl::fz_post_k(P, Mdl::fz_pre_lite(P, c, kk), z, n0, kk);
        const float z1 = Mdl::fz_post_k(P, Mdl::fz_pre_lite(P, c, kk + 1), z, n1, kk + 1);
        pj.add(ca[kk / 2], z0, z1);
      });
  return pj.logpy(P, yrow);
}

// lam + g as a separate rounding: g is opaque to the compiler, so no
// multiply inside it is fused into this add (the weights kernel and the
// new-cloud kernel, which adds lam later, get the same bits).
__device__ __forceinline__ float la_ell(float lam, float g) {
  asm volatile("" : "+v"(g));
  return lam + g;
}
template <class Mdl, int SEG, int JPT>
__device__ __forceinline__ void la_weights_tile(const StepArgs& a, int ti, bool fallback) {
  __shared__ SegScratch sh;
  const int4 tile = a.tiles[ti];
  const int f = tile.x;
  const int am = a.active != nullptr ? a.active[f] : 1;
  const int tf = a.run_Tf != nullptr ? a.run_Tf[f] : 0x7fffffff;
  asm volatile("" ::"v"(am), "v"(tf));
  const FilterView fv = load_filter(a, f);
  const bool act = am != 0 && fv.t < min(tf, a.run_T);  // step_active
  if (!fallback && tile.z == 0 && threadIdx.x == 0) a.act[f] = act ? 1 : 0;
  if (!act) return;
  const int N = fv.N, M = fv.M;
  const int i = tile.y + threadIdx.x / SEG;
  const int ls = threadIdx.x % SEG;
  const bool vi = i < N;
  const int oo = fv.oo;
  const long long io = fv.io;
  const int t = fv.t + 1;
  const unsigned char cb = (unsigned char)fv.cur;
  const int src = copy_of(cb);
  const Key key = make_key(a.seed, (uint32_t)f);
  const int ci = vi ? (ident_slots(cb, src) ? i : a.ind[src][oo + i]) : 0;

  float y[Mdl::DY], x[Mdl::DX];
  load_y<Mdl>(a, f, t, y);
#pragma unroll
  for (int d = 0; d < Mdl::DX; ++d) x[d] = vi ? a.x[src][(long long)d * a.NT + oo + i] : 0.f;

  const float* zrow = a.z[src] + (io + (long long)ci * M) * Mdl::DZ;
  const float* lrow = a.lam[src] + io + (long long)ci * M;
  float* erow = a.ell + io + (long long)(vi ? i : 0) * M;
  Lse acc;
  constexpr bool kH = has_yhat<Mdl>();
  const bool want_h = kH && a.yp != nullptr && !fallback;
  float hv = 0.f;  // sum over the lane's draws of qbar h(xla, zla)
  if constexpr (Mdl::kStreamZ) {
    // wide z: every lane of the wave takes part in the matrix-core residual
    float ca[WaveProj<Mdl>::NA];
    WaveProj<Mdl>::load_a(as_prm(a.prm), ca);
    const float* yrow = y_row<Mdl>(a, f, t);
    for (int r = 0; r < JPT; ++r) {
      const int j = ls + r * SEG;
      const bool on = vi && j < M;
      float z[Mdl::DZ];
#pragma unroll
      for (int d = 0; d < Mdl::DZ; ++d) z[d] = on ? zrow[d * M + j] : 0.f;
      const float lj = on ? lrow[j] : 0.f;
      const float g = la_logpy_wave<Mdl>(a, key, t, i, on ? j : 0, x, z, yrow, ca);
      if (on) {
        const float e = la_ell(lj, g);
        erow[j] = e;
        acc.add(e);
      }
    }
  } else {
#pragma unroll
  for (int r = 0; r < JPT; ++r) {
    const int j = ls + r * SEG;
    if (vi && j < M) {
      float z[Mdl::DZ];
#pragma unroll
      for (int d = 0; d < Mdl::DZ; ++d) z[d] = zrow[d * M + j];
      const float lj = lrow[j];
      float g;
      if (want_h) {
        float h[1];
        g = la_logpy<Mdl, kH>(a, key, t, i, j, x, z, y, h);
        hv += fast_exp(lj) * h[0];
      } else {
        g = la_logpy<Mdl>(a, key, t, i, j, x, z, y);
      }
      const float e = la_ell(lj, g);
      erow[j] = e;
      acc.add(e);
    }
  }
  }
  const float lw = seg_lse<SEG>(acc, sh);
  if (vi && ls == 0) a.logw[oo + i] = lw;
  if (want_h) {
    const float hs = seg_sum<SEG>(hv, sh);
    if (vi && ls == 0) a.yp[oo + i] = hs;
  }
}

// Nested look-ahead weights (Fig. 4 step 1 with N_z' = K companions per
// candidate, eq:weightsMC): candidate m of outer particle i is drawn from
// inner component m as in the paired form (LA_X at (t, i, m)); its K
// companions take ancestors by systematic resampling (U53 LA_B at
// (t, i, m)) of the inner weights conditioned on the candidate,
// kappa_j = lam_j + log p(xla_m | x_i, z_j) (eq:qnobar), and are propagated
// with the inner prior (LA_Z normals k dz .. k dz + dz - 1 at (t, i, m));
// ell_m = lam_m + log (1/K) sum_k p(y_t | xla_m, zla_mk).  When p(x' | x, z)
// does not depend on z the conditioned weights are lam itself: one
// cumulative sum serves every candidate and each lane scores its own
// candidates.  Otherwise the segment walks the candidates in order, forming
// each one's conditioned cumulative sum together and spreading its
// companions over the lanes.
template <class Mdl, int SEG, int JPT>
__device__ __forceinline__ void la_weights_nested_tile(const StepArgs& a, int ti) {
  constexpr int DX = Mdl::DX, DZ = Mdl::DZ, DY = Mdl::DY;
  constexpr int NSEG = kBlock / SEG, CAP = SEG * JPT;
  constexpr bool kCond = Mdl::kXdepZ;
  constexpr bool kHoldZ = kCond && JPT * DZ <= 64;  // the lane's cloud stays in registers
  __shared__ SegScratch sh;
  __shared__ double cdf[NSEG][kCond ? 1 : CAP];
  __shared__ float cz[NSEG][kCond ? CAP : 1][DZ];
  __shared__ float lms[NSEG][kCond ? CAP : 1];
  // each lane's conditioned weights of its current candidate, kept between
  // the total and the cumulative pass when the cloud is small (row padded
  // by one word: lanes at the same index fall in different banks)
  constexpr bool kWCache = kCond && CAP <= 32;
  __shared__ float wc[kWCache ? kBlock : 1][kWCache ? CAP + 1 : 1];
  constexpr bool kH = has_yhat<Mdl>();
  const int4 tile = a.tiles[ti];
  const int f = tile.x;
  const int am = a.active != nullptr ? a.active[f] : 1;
  const int tf = a.run_Tf != nullptr ? a.run_Tf[f] : 0x7fffffff;
  asm volatile("" ::"v"(am), "v"(tf));
  const FilterView fv = load_filter(a, f);
  const bool act = am != 0 && fv.t < min(tf, a.run_T);  // step_active
  if (tile.z == 0 && threadIdx.x == 0) a.act[f] = act ? 1 : 0;
  if (!act) return;
  const int N = fv.N, M = fv.M, K = a.n_comp;
  constexpr int CPB = comp_per_block<DZ>();  // companions per block of normals
  const int s = threadIdx.x / SEG;
  const int i = tile.y + s;
  const int ls = threadIdx.x % SEG;
  const bool vi = i < N;
  const int oo = fv.oo;
  const long long io = fv.io;
  const int t = fv.t + 1;
  const unsigned char cb = (unsigned char)fv.cur;
  const int src = copy_of(cb);
  const Key key = make_key(a.seed, (uint32_t)f);
  const int ci = vi ? (ident_slots(cb, src) ? i : a.ind[src][oo + i]) : 0;
  const float logK = fast_log((float)K);

  float y[DY], x[DX];
  load_y<Mdl>(a, f, t, y);
#pragma unroll
  for (int d = 0; d < DX; ++d) x[d] = vi ? a.x[src][(long long)d * a.NT + oo + i] : 0.f;
  const float* zrow = a.z[src] + (io + (long long)ci * M) * DZ;
  const float* lrow = a.lam[src] + io + (long long)ci * M;
  float* erow = a.ell + io + (long long)(vi ? i : 0) * M;

  // candidates (as in the paired form) and the lanes' inner weights
  float lamv[JPT], xl[JPT][DX];
  float zh[kHoldZ ? JPT : 1][kHoldZ ? DZ : 1];
#pragma unroll
  for (int r = 0; r < JPT; ++r) {
    const int j = ls + r * SEG;
    lamv[r] = -INFINITY;
#pragma unroll
    for (int d = 0; d < DX; ++d) xl[r][d] = 0.f;
    if (vi && j < M) {
      float z[DZ], nu[DX];
#pragma unroll
      for (int d = 0; d < DZ; ++d) z[d] = zrow[d * M + j];
      if constexpr (kHoldZ) {
#pragma unroll
        for (int d = 0; d < DZ; ++d) zh[kHoldZ ? r : 0][kHoldZ ? d : 0] = z[d];
      }
      lamv[r] = lrow[j];
      normals<DX>(key, (uint32_t)t, (uint32_t)i, (uint32_t)j, P_LA_X, nu);
      Mdl::fx(as_prm(a.prm), x, z, nu, t - 1, xl[r]);
      if constexpr (kCond) lms[s][kCond ? j : 0] = lamv[r];
    }
  }
  // predicted observation: sum over the lane's candidates of qbar times the
  // mean of h over their companions
  const bool want_h = kH && a.yp != nullptr;
  const float invK = 1.0f / (float)K;
  float hv = 0.f;
  float ev[JPT];
#pragma unroll
  for (int r = 0; r < JPT; ++r) ev[r] = -INFINITY;

  if constexpr (!kCond) {
    // ---- one cumulative sum of the inner weights for every candidate
    float mloc = -INFINITY;
#pragma unroll
    for (int r = 0; r < JPT; ++r)
      if (finitef(lamv[r])) mloc = fmaxf(mloc, lamv[r]);
    const float m0 = seg_max<SEG>(mloc, sh);
    const bool deg = !(m0 > -INFINITY);
    double carry = 0.0;
#pragma unroll
    for (int r = 0; r < JPT; ++r) {
      const int j = ls + r * SEG;
      double w = 0.0;
      if (j < M) w = deg ? 1.0 : (finitef(lamv[r]) ? (double)fast_exp(lamv[r] - m0) : 0.0);
      double tot;
      const double c = seg_scan_incl<SEG>(w, sh, tot);
      cdf[s][r * SEG + ls] = carry + c;
      carry += tot;
    }
    seg_lds_sync<SEG>();
    const double total = cdf[s][M - 1];
#pragma unroll
    for (int r = 0; r < JPT; ++r) {
      const int j = ls + r * SEG;
      if (vi && j < M) {
        float pre[Mdl::NPRE], r0[DY];
        Mdl::fz_pre(as_prm(a.prm), x, xl[r], t - 1, pre);
        Mdl::obs_pre(as_prm(a.prm), y, xl[r], r0);
        const double u = uniform53_ab(key, (uint32_t)t, (uint32_t)i, (uint32_t)j, P_LA_B);
        Lse acck;
        float hk = 0.f;
        for (int k0 = 0; k0 < K; k0 += CPB) {
          float nb[CPB * DZ];
          normals_kb<DZ>(key, (uint32_t)t, (uint32_t)i, (uint32_t)j, P_LA_Z, k0, nb);
#pragma unroll
          for (int q = 0; q < CPB; ++q) {
            const int k = k0 + q;
            if (k >= K) break;
            const int b = cdf_search(cdf[s], M, sys_point(k, u, total, K));
            float zg[DZ], zc[DZ];
#pragma unroll
            for (int d = 0; d < DZ; ++d) zg[d] = zrow[d * M + b];
            Mdl::fz_post(as_prm(a.prm), pre, zg, nb + q * DZ, zc);
            acck.add(Mdl::logpy_post(as_prm(a.prm), r0, zc));
            if constexpr (kH) {
              if (want_h) {
                float h[1];
                Mdl::obs_mean(as_prm(a.prm), xl[r], zc, h);
                hk += h[0];
              }
            }
          }
        }
        const float g = (acck.m == -INFINITY) ? -INFINITY : acck.m + fast_log(acck.s) - logK;
        ev[r] = la_ell(lamv[r], g);
        if (want_h) hv += fast_exp(lamv[r]) * (hk * invK);
      }
    }
  } else {
    // ---- each lane scores its own candidates.  Per candidate, three passes
    // over the segment's cloud (staged in LDS, read by every lane at the same
    // index): the largest conditioned log-weight, the FP64 total, then the
    // cumulative sum in inner order up to each systematic point (companion k
    // takes the first index whose cumulative weight exceeds point k; points
    // at or past the total take the last index with positive weight).
#pragma unroll
    for (int r = 0; r < JPT; ++r) {
      const int j = ls + r * SEG;
      if (j < M) {
#pragma unroll
        for (int d = 0; d < DZ; ++d)
          cz[s][kCond ? j : 0][d] = vi ? (kHoldZ ? zh[kHoldZ ? r : 0][kHoldZ ? d : 0] : zrow[d * M + j]) : 0.f;
      }
    }
    seg_lds_sync<SEG>();
    if (vi) {
#pragma unroll
      for (int r = 0; r < JPT; ++r) {
        const int j = ls + r * SEG;
        if (j >= M) continue;
        // conditioned log-weight of inner particle jj given this candidate
        float cpx[Mdl::NPX];
        Mdl::px_pre(as_prm(a.prm), xl[r], x, t - 1, cpx);
        auto kappa = [&](int jj) {
          float zj[DZ];
#pragma unroll
          for (int d = 0; d < DZ; ++d) zj[d] = cz[s][kCond ? jj : 0][d];
          float kp = lms[s][kCond ? jj : 0] + Mdl::logpx_post(as_prm(a.prm), cpx, zj);
          asm volatile("" : "+v"(kp));
          return kp;
        };
        float mx = -INFINITY;
        for (int jj = 0; jj < M; ++jj) {
          const float kp = kappa(jj);
          if (finitef(kp)) mx = fmaxf(mx, kp);
        }
        const bool deg = !(mx > -INFINITY);
        auto weight = [&](int jj) -> float {
          const float kp = kappa(jj);
          return deg ? 1.0f : (finitef(kp) ? fast_exp(kp - mx) : 0.0f);
        };
        double total = 0.0;
        int lastpos = 0;
        for (int jj = 0; jj < M; ++jj) {
          const float w = weight(jj);
          if constexpr (kWCache) wc[kWCache ? threadIdx.x : 0][kWCache ? jj : 0] = w;
          total += (double)w;
          if (w > 0.0f) lastpos = jj;
        }
        // the third pass takes these weights back (small clouds) or forms
        // them again, the same values either way
        auto weight3 = [&](int jj) -> double {
          if constexpr (kWCache) return (double)wc[kWCache ? threadIdx.x : 0][kWCache ? jj : 0];
          else return (double)weight(jj);
        };
        const double u = uniform53_ab(key, (uint32_t)t, (uint32_t)i, (uint32_t)j, P_LA_B);
        float pre[Mdl::NPRE], r0[DY];
        Mdl::fz_pre(as_prm(a.prm), x, xl[r], t - 1, pre);
        Mdl::obs_pre(as_prm(a.prm), y, xl[r], r0);
        Lse acck;
        float hk = 0.f;
        auto emit = [&](int b, const float* nu) {
          float zg[DZ], zc[DZ];
#pragma unroll
          for (int d = 0; d < DZ; ++d) zg[d] = cz[s][kCond ? b : 0][d];
          Mdl::fz_post(as_prm(a.prm), pre, zg, nu, zc);
          acck.add(Mdl::logpy_post(as_prm(a.prm), r0, zc));
          if constexpr (kH) {
            if (want_h) {
              float h[1];
              Mdl::obs_mean(as_prm(a.prm), xl[r], zc, h);
              hk += h[0];
            }
          }
        };
        // companion k: a cursor over the cumulative sum advances to the
        // first index whose sum exceeds point k (the points increase), then
        // every lane propagates its companion k together
        int jc = -1;
        double c = 0.0;
        for (int k0 = 0; k0 < K; k0 += CPB) {
          float nb[CPB * DZ];
          normals_kb<DZ>(key, (uint32_t)t, (uint32_t)i, (uint32_t)j, P_LA_Z, k0, nb);
#pragma unroll
          for (int q = 0; q < CPB; ++q) {
            const int k = k0 + q;
            if (k >= K) break;
            const double P = sys_point(k, u, total, K);
            while (!(c > P) && jc + 1 < M) {
              ++jc;
              c += weight3(jc);
            }
            emit(c > P ? jc : lastpos, nb + q * DZ);
          }
        }
        const float g = (acck.m == -INFINITY) ? -INFINITY : acck.m + fast_log(acck.s) - logK;
        ev[r] = la_ell(lamv[r], g);
        if (want_h) hv += fast_exp(lamv[r]) * (hk * invK);
      }
    }
  }
  Lse acc;
#pragma unroll
  for (int r = 0; r < JPT; ++r) {
    const int j = ls + r * SEG;
    if (vi && j < M) {
      erow[j] = ev[r];
      acc.add(ev[r]);
    }
  }
  const float lw = seg_lse<SEG>(acc, sh);
  if (vi && ls == 0) a.logw[oo + i] = lw;
  if (want_h) {
    const float hs = seg_sum<SEG>(hv, sh);
    if (vi && ls == 0) a.yp[oo + i] = hs;
  }
}

template <class Mdl, int SEG, int JPT>
__global__ __launch_bounds__(kBlock) void k_la_weights_nested(StepArgs a) {
  la_weights_nested_tile<Mdl, SEG, JPT>(a, blockIdx.x);
}

static __device__ bool learned_rejected(const StepArgs& a, int f, int N, float* fred4, double* red4);

// One workgroup per tile.  (A kernel that loops over tiles compiles to
// markedly slower code for the single-tile case, so the learned step's
// fallback has kernels of its own.)
template <class Mdl, int SEG, int JPT>
static __global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(min_waves<Mdl>()))) void k_la_weights(StepArgs a) {
  la_weights_tile<Mdl, SEG, JPT>(a, blockIdx.x, false);
}

// Learned step's fallback, a smaller grid looping over the tiles: each
// workgroup loads its tiles' filters at once, decides per filter whether the
// learned proposals are rejected (the workgroup holding a filter's first
// tile records the decision and the fallback flag), and runs the look-ahead
// weights only for the tiles of rejecting filters.
template <class Mdl, int SEG, int JPT>
static __global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(min_waves<Mdl>()))) void k_la_weights_fallback(StepArgs a) {
  __shared__ int tfl[kBlock], runs[kBlock], todo[kBlock], wcnt[kBlock / kWave];
  __shared__ unsigned char rejr[kBlock];
  __shared__ float fred4[kBlock / kWave];
  __shared__ double red4[kBlock / kWave];
  const int th = threadIdx.x;
  for (int base = blockIdx.x; base < a.n_tiles; base += kBlock * gridDim.x) {
    const int mine = base + th * gridDim.x;
    const bool have = mine < a.n_tiles;
    const int4 tl = have ? a.tiles[mine] : make_int4(-1, 0, 0, 0);
    tfl[th] = tl.x;
    __syncthreads();
    // runs of equal filters (tiles are ordered by filter within a class)
    const bool start = have && (th == 0 || tfl[th - 1] != tl.x);
    int myrun;
    const int nr = block_compact(start, th, runs, wcnt, &myrun);
    for (int r = 0; r < nr; ++r) {
      const int f = tfl[runs[r]];
      const bool rej = step_active(a, f) && learned_rejected(a, f, a.fN[f], fred4, red4);
      if (th == 0) rejr[r] = rej ? 1 : 0;
      __syncthreads();
    }
    const bool rj = have && rejr[myrun - 1] != 0;
    if (have && tl.z == 0) {
      a.fb[tl.x] = rj ? 1 : 0;
      if (rj) {
        atomicOr(&a.flags[tl.x], (uint32_t)F_FALLBACK);
        a.lflags[tl.x] = 0u;
      }
    }
    const int nt = block_compact(rj, mine, todo, wcnt, nullptr);
    for (int q = 0; q < nt; ++q) {
      la_weights_tile<Mdl, SEG, JPT>(a, todo[q], true);
      __syncthreads();
    }
  }
}

// --------------------------------------------------------- plain weights
// Fig. 2 step 1 (eq:approx2 with unit inner weights): ell = log p(y_t | xt, zt),
// log w_i = logsumexp_j ell - log M, and the per-particle partial
// sum_j qbar_ij zt_ij (qbar = softmax_j ell, step 3) for the estimate.
template <class Mdl, int SEG, int JPT>
static __global__ __launch_bounds__(kBlock) void k_dpf_weights(StepArgs a) {
  __shared__ SegScratch sh;
  __shared__ float vred[kBlock / kWave][Mdl::DZ];
  const int4 tile = a.tiles[blockIdx.x];
  const int f = tile.x;
  const bool act = step_active(a, f);
  if (tile.z == 0 && threadIdx.x == 0) a.act[f] = act ? 1 : 0;
  if (!act) return;
  const int N = a.fN[f], M = a.fM[f];
  const int i = tile.y + threadIdx.x / SEG;
  const int ls = threadIdx.x % SEG;
  const bool vi = i < N;
  const int oo = a.ooff[f];
  const long long io = a.ioff[f];
  const int t = a.tcur[f] + 1;
  const int src = copy_of(a.cur[f]);

  float y[Mdl::DY], x[Mdl::DX], r0[Mdl::DY];
  load_y<Mdl>(a, f, t, y);
#pragma unroll
  for (int d = 0; d < Mdl::DX; ++d) x[d] = vi ? a.x[src][(long long)d * a.NT + oo + i] : 0.f;
  Mdl::obs_pre(as_prm(a.prm), y, x, r0);
  const float* zrow = a.z[src] + (io + (long long)(vi ? i : 0) * M) * Mdl::DZ;
  float* erow = a.ell + io + (long long)(vi ? i : 0) * M;
  float ev[JPT];
  Lse acc;
#pragma unroll
  for (int r = 0; r < JPT; ++r) {
    const int j = ls + r * SEG;
    ev[r] = -INFINITY;
    if (vi && j < M) {
      float z[Mdl::DZ];
#pragma unroll
      for (int d = 0; d < Mdl::DZ; ++d) z[d] = zrow[d * M + j];
      ev[r] = Mdl::logpy_post(as_prm(a.prm), r0, z);
      erow[j] = ev[r];
      acc.add(ev[r]);
    }
  }
  const float lse = seg_lse<SEG>(acc, sh);
  // qbar-weighted cloud mean of the proposals (uniform if degenerate)
  const bool deg = !(lse > -INFINITY);
  float part[Mdl::DZ];
#pragma unroll
  for (int d = 0; d < Mdl::DZ; ++d) part[d] = 0.f;
#pragma unroll
  for (int r = 0; r < JPT; ++r) {
    const int j = ls + r * SEG;
    if (vi && j < M) {
      const float q = deg ? 1.0f / (float)M : (finitef(ev[r]) ? fast_exp(ev[r] - lse) : 0.f);
#pragma unroll
      for (int d = 0; d < Mdl::DZ; ++d) part[d] += q * zrow[d * M + j];
    }
  }
  const float lw = deg ? -INFINITY : lse - fast_log((float)M);
  float* kp = a.kpart + (long long)(oo + i) * Mdl::DZ;
  if constexpr (Mdl::DZ <= 16) {
    int slot;
    const float tot = seg_sum_vec_t<SEG, Mdl::DZ>(part, vred, slot);
    if (vi && slot >= 0) kp[slot] = tot;
  } else {
    seg_sum_vec<SEG, Mdl::DZ>(part, vred);
    if (vi && ls == 0) {
#pragma unroll
      for (int d = 0; d < Mdl::DZ; ++d) kp[d] = part[d];
    }
  }
  if (vi && ls == 0) {
    a.logw[oo + i] = lw;
    if (deg) atomicOr(&a.flags[f], (uint32_t)F_DEGENERATE_INNER);
  }
}

// -------------------------------------------------------- outer resampling
// Systematic resampling of the N outer weights w_i = exp(log w_i - max)
// (Fig. 4 step 3; Fig. 2 step 2), organised around groups of 256 weights.
// Group g carries its own shift m_g = max of its log-weights, the FP64 sum
// s_g of exp(log w_i - m_g) and the sum of squares q_g (one workgroup per
// group, k_res_stats).  A workgroup that needs ancestors combines the
// statistics -- m = max_g m_g, c_g = exp(m_g - m), T_g = c_g s_g, offsets
// B_g = inclusive scan of T -- always with the same code in the same order,
// so every workgroup agrees bit for bit on them; group g's cumulative weights
// are C_i = min(B_g + c_g L_i, B_{g+1}) (L: inclusive FP64 scan of its
// terms), its last one B_{g+1}: monotone, with shared boundaries.  A
// systematic point ((k + u) C_total) / N lies in the first group with
// B_{g+1} > point and takes the first index there with C_i > point (a point
// at or past the total takes the first index reaching the total).  The new
// particles' workgroups resolve their own ancestors this way, so no
// separate selection launch is needed.

// Log-weight source: FP32 log-weights, FP32 exponent of the shifted value.
struct LogSrc {
  const float* lw;
  static constexpr bool kLog = true;
  __device__ float key(int i) const {
    const float v = lw[i];
    return finitef(v) ? v : -INFINITY;
  }
  __device__ double val(int i, float mg) const {
    const float v = lw[i];
    return finitef(v) ? (double)fast_exp(v - mg) : 0.0;
  }
};

// Linear FP64 weights as given (kernel-level primitive).
struct LinSrc {
  const double* w;
  static constexpr bool kLog = false;
  __device__ float key(int) const { return 0.f; }
  __device__ double val(int i, float) const { return w[i]; }
};

__device__ __forceinline__ float block_max_256(float v, float* red4) {
  v = seg_reduce_wave<OpMax, kWave>(v);
  if ((threadIdx.x & (kWave - 1)) == 0) red4[threadIdx.x / kWave] = v;
  __syncthreads();
  const float r = fmaxf(fmaxf(red4[0], red4[1]), fmaxf(red4[2], red4[3]));
  __syncthreads();
  return r;
}

// Scale of group g relative to the global shift, exp(m_g - m) in (0, 1]
// (FP32 exponent widened; every workgroup evaluates it identically).
template <class Src>
__device__ __forceinline__ double group_scale(float mg, float m) {
  if (!Src::kLog) return 1.0;
  return mg > -INFINITY ? (double)fast_exp(mg - m) : 0.0;
}

// Learned step: whether filter f rejects its learned proposals -- no finite
// log-weight, or ESS = (sum w)^2 / sum w^2 below ess_frac * N -- from the
// group statistics of the learned log-weights.  All 256 threads take part;
// every workgroup gets the same answer.
static __device__ bool learned_rejected(const StepArgs& a, int f, int N, float* fred4, double* red4) {
  const int th = threadIdx.x;
  const int G = a.finfo[f].ngroup;
  const double* gs = a.gstat + 4LL * a.finfo[f].rg_base;
  // the three statistics of a group in one memory round (clamped, masked)
  const int thc = min(th, G - 1);
  const double g0 = gs[4 * thc], g1 = gs[4 * thc + 1], g2 = gs[4 * thc + 2];
  const float gm = th < G ? (float)g0 : -INFINITY;
  const float m = block_max_256(gm, fred4);
  if (!(m > -INFINITY)) return true;
  double T = 0.0, Q = 0.0;
  if (th < G) {
    const double c = group_scale<LogSrc>(gm, m);
    T = c * g1;
    Q = (c * c) * g2;
  }
  const double total = block_sum_256(T, red4);
  const double sumsq = block_sum_256(Q, red4);
  return total * total < a.ess_frac * (double)N * sumsq;
}

struct ResScratch {
  double B[kBlock + 1];   // group offsets (at most 256 groups)
  double C[kResGroup];    // cumulative weights of the group being resolved
  double P[kBlock];       // points of this workgroup
  int gsel[kBlock];       // their groups
  int run0[kBlock];       // first point of each run of points sharing a group
  int wcnt[kBlock / kWave];
  double red4[kBlock / kWave];
  float fred4[kBlock / kWave];
};

// Statistics (m_g, s_g, q_g) of group g.
template <class Src>
__device__ void res_group_stat(const Src& src, int n, int g, float& mg, double& sg, double& qg,
                               ResScratch& sh) {
  const int i = g * kResGroup + threadIdx.x;
  const float key = i < n ? src.key(i) : -INFINITY;
  mg = Src::kLog ? block_max_256(key, sh.fred4) : 0.f;
  const double v = (i < n && (!Src::kLog || mg > -INFINITY)) ? src.val(i, mg) : 0.0;
  sg = block_sum_256(v, sh.red4);
  qg = block_sum_256(v * v, sh.red4);
}

// The same from this thread's log-weight lw already loaded (valid: i < n),
// with the same arithmetic as for LogSrc.
__device__ __forceinline__ void res_group_stat_lw(float lw, bool valid, float& mg, double& sg, double& qg,
                                                  ResScratch& sh) {
  const float key = valid && finitef(lw) ? lw : -INFINITY;
  mg = block_max_256(key, sh.fred4);
  const double v = (valid && mg > -INFINITY) ? (finitef(lw) ? (double)fast_exp(lw - mg) : 0.0) : 0.0;
  sg = block_sum_256(v, sh.red4);
  qg = block_sum_256(v * v, sh.red4);
}

struct ResResult {
  float m;       // max log-weight (0 for linear weights or when degenerate)
  double total;  // sum of the weights exp(log w - m)
  double sumsq;  // sum of their squares
  bool deg;      // no finite log-weight: uniform weights were used
};

// Ancestors res[j] of the points k0 + j, j < np (np <= 256), from the G group
// statistics gstat [G][4] (m_g, s_g, q_g, -).  want_sumsq: also return the
// sum of squared weights (for the effective sample size).
template <class Src>
__device__ ResResult resolve_points(const Src& src, int n, int n_out, double u, int k0, int np,
                                    const double* gstat, int G, int* res, ResScratch& sh, bool want_sumsq) {
  const int th = threadIdx.x;
  const float gm_t = th < G ? (float)gstat[4 * th] : -INFINITY;
  const float m = Src::kLog ? block_max_256(gm_t, sh.fred4) : 0.f;
  const bool deg = Src::kLog && !(m > -INFINITY);
  double T = 0.0, Q = 0.0;
  if (th < G) {
    if (deg) {
      T = Q = (double)min(kResGroup, n - th * kResGroup);
    } else {
      const double c = group_scale<Src>(gm_t, m);
      T = c * gstat[4 * th + 1];
      Q = (c * c) * gstat[4 * th + 2];
    }
  }
  sh.B[th + 1] = block_scan_incl_256(T, sh.red4);  // its barriers order the writes below
  if (th == 0) sh.B[0] = 0.0;
  const double sumsq = want_sumsq ? block_sum_256(Q, sh.red4) : 0.0;
  __syncthreads();
  const double total = sh.B[G];
  if (th < np) {
    const double P = sys_point(k0 + th, u, total, n_out);
    int lo = 0, hi = G;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (sh.B[mid + 1] > P)
        hi = mid;
      else
        lo = mid + 1;
    }
    if (lo == G) {
      lo = 0;
      hi = G - 1;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (sh.B[mid + 1] >= total)
          hi = mid;
        else
          lo = mid + 1;
      }
    }
    sh.P[th] = P;
    sh.gsel[th] = lo;
  }
  __syncthreads();
  // points are non-decreasing, so their groups are too: list the runs of
  // points per group and visit each distinct group once (few points: a
  // scan by every thread; many: ranks of the run starts by compaction)
  int nruns;
  if (np <= 16) {
    nruns = 0;
    for (int j = 0; j < np; ++j)
      if (j == 0 || sh.gsel[j] != sh.gsel[j - 1]) {
        if (th == 0) sh.run0[nruns] = j;
        ++nruns;
      }
    __syncthreads();
  } else {
    const bool start = th < np && (th == 0 || sh.gsel[th - 1] != sh.gsel[th]);
    nruns = block_compact(start, th, sh.run0, sh.wcnt, nullptr);
  }
  for (int r = 0; r < nruns; ++r) {
    const int j0 = sh.run0[r];
    const int j1 = r + 1 < nruns ? sh.run0[r + 1] : np;
    const int g = sh.gsel[j0];
    const int base = g * kResGroup;
    const int nloc = min(kResGroup, n - base);
    const float mg = Src::kLog ? (float)gstat[4 * g] : 0.f;
    const double cg = deg ? 1.0 : group_scale<Src>(mg, m);
    double v = 0.0;
    if (th < nloc) v = deg ? 1.0 : ((!Src::kLog || mg > -INFINITY) ? src.val(base + th, mg) : 0.0);
    const double L = block_scan_incl_256(v, sh.red4);
    const double Bg = sh.B[g], Bg1 = sh.B[g + 1];
    if (th < nloc) sh.C[th] = (th == nloc - 1) ? Bg1 : fmin(Bg + cg * L, Bg1);
    __syncthreads();
    if (th >= j0 && th < j1) res[th] = base + cdf_search(sh.C, nloc, sh.P[th]);
    __syncthreads();
  }
  ResResult r;
  r.m = deg ? 0.f : m;
  r.total = total;
  r.sumsq = sumsq;
  r.deg = deg;
  return r;
}

// ------------------------------------------------ wave-level draws (wave 0)
// When a workgroup serves one outer particle, its ancestor and candidate are
// single draws: one wave does them with wave-wide DPP scans (no LDS rounds,
// no barriers) while the other waves get on with independent work.

// Inclusive FP64 scan over the 64 lanes; excl receives the exclusive value.
__device__ __forceinline__ double wave_scan_d(double v, double& excl) {
  const double incl = seg_scan_wave<kWave>(v);
  const double up = __shfl_up(incl, 1);
  excl = (threadIdx.x & (kWave - 1)) == 0 ? 0.0 : up;
  return incl;
}

__device__ __forceinline__ int first_lane(unsigned long long mask) { return __ffsll((long long)mask) - 1; }

// The ancestor of point k0 (one systematic point) from the group statistics
// (lane l holds group l's (m, s, q) in gs), by one wave; G <= 64.  Same rule
// and group offsets B as resolve_points (whose wave 0 computes B with the
// same scan); the group's cumulative weights are summed four per lane then
// scanned across lanes.
template <class Src>
__device__ int resolve_point_w0(const Src& src, int n, int n_out, double u, int k0, const double* gs, int G,
                                bool want_sumsq, ResResult& rr) {
  const int l = threadIdx.x & (kWave - 1);
  const float gm = l < G ? (float)gs[0] : -INFINITY;
  const float m = Src::kLog ? seg_reduce_wave<OpMax, kWave>(gm) : 0.f;
  const bool deg = Src::kLog && !(m > -INFINITY);
  double T = 0.0, Q = 0.0;
  if (l < G) {
    if (deg) {
      T = Q = (double)min(kResGroup, n - l * kResGroup);
    } else {
      const double c = group_scale<Src>(gm, m);
      T = c * gs[1];
      Q = (c * c) * gs[2];
    }
  }
  const double Binc = seg_scan_wave<kWave>(T);  // B[l + 1]
  const double total = readlane_d(Binc, G - 1);
  rr.m = deg ? 0.f : m;
  rr.total = total;
  rr.sumsq = want_sumsq ? seg_reduce_wave<OpAdd, kWave>(Q) : 0.0;
  rr.deg = deg;
  const double P = sys_point(k0, u, total, n_out);
  unsigned long long bm = __ballot(l < G && Binc > P);
  if (!bm) bm = __ballot(l < G && Binc >= total);
  const int g = first_lane(bm);
  const int base = g * kResGroup;
  const int nloc = min(kResGroup, n - base);
  const float mg = Src::kLog ? __int_as_float(__builtin_amdgcn_readlane(__float_as_int(gm), g)) : 0.f;
  const double cg = deg ? 1.0 : group_scale<Src>(mg, m);
  const double Bg = g > 0 ? readlane_d(Binc, g - 1) : 0.0;
  const double Bg1 = readlane_d(Binc, g);
  // the four weights are read at clamped indices first (loads in flight
  // together; a guarded load would wait inside its own branch), then masked
  double L[4], vv[4], acc = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = 4 * l + q;
    vv[q] = src.val(base + (i < nloc ? i : 0), mg);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = 4 * l + q;
    const double v = i < nloc ? (deg ? 1.0 : ((!Src::kLog || mg > -INFINITY) ? vv[q] : 0.0)) : 0.0;
    acc += v;
    L[q] = acc;
  }
  double ex;
  wave_scan_d(acc, ex);
  double C[4];
  int hit = 4, hit_eq = 4;
#pragma unroll
  for (int q = 3; q >= 0; --q) {
    const int i = 4 * l + q;
    C[q] = (i == nloc - 1) ? Bg1 : fmin(Bg + cg * (ex + L[q]), Bg1);
    if (i < nloc && C[q] > P) hit = q;
    if (i < nloc && C[q] >= Bg1) hit_eq = q;
  }
  bm = __ballot(hit < 4);
  int idx;
  if (bm) {
    const int fl = first_lane(bm);
    idx = 4 * fl + __builtin_amdgcn_readlane(hit, fl);
  } else {
    const int fl = first_lane(__ballot(hit_eq < 4));
    idx = 4 * fl + __builtin_amdgcn_readlane(hit_eq, fl);
  }
  return base + idx;
}

// One systematic draw (offset u) over weights exp(e_j - max), j < M (non-
// finite: 0; none finite: uniform), by one wave: each lane sums a chunk of
// ceil(M / 64) <= CMAX consecutive weights, the chunk totals are scanned
// across lanes, and the lane holding the point walks its chunk.  Chunks of
// up to 16 stay in registers; longer ones are read again.
template <int CMAX>
__device__ int select_w0(const float* e, int M, double u, bool& deg_out) {
  constexpr bool kReg = CMAX <= 16;
  constexpr int R = kReg ? CMAX : 1;
  const int l = threadIdx.x & (kWave - 1);
  const int C = (M + kWave - 1) / kWave;
  const int j0 = l * C;
  const int nv = max(0, min(C, M - j0));  // entries of this lane's chunk
  float ev[R];
  float mloc = -INFINITY;
  if constexpr (kReg) {
#pragma unroll
    for (int q = 0; q < R; ++q) {
      ev[q] = q < nv ? e[j0 + q] : -INFINITY;
      if (finitef(ev[q])) mloc = fmaxf(mloc, ev[q]);
    }
  } else {
    for (int q = 0; q < nv; ++q) {
      const float v = e[j0 + q];
      if (finitef(v)) mloc = fmaxf(mloc, v);
    }
  }
  const float m = seg_reduce_wave<OpMax, kWave>(mloc);
  const bool deg = !(m > -INFINITY);
  deg_out = deg;
  auto wt = [&](float v) { return deg ? 1.0 : (finitef(v) ? (double)fast_exp(v - m) : 0.0); };
  double acc = 0.0;
  double wv[R];
  if constexpr (kReg) {
#pragma unroll
    for (int q = 0; q < R; ++q) {
      wv[q] = q < nv ? wt(ev[q]) : 0.0;
      acc += wv[q];
    }
  } else {
    for (int q = 0; q < nv; ++q) acc += wt(e[j0 + q]);
  }
  double ex;
  const double incl = wave_scan_d(acc, ex);
  const double total = readlane_d(incl, (M - 1) / C);  // the last lane with entries
  const double P = sys_point(0, u, total, 1);
  // the first lane with entries whose cumulative weight passes the point
  // (else reaches the total); its last entry's cumulative weight is its
  // scanned value, so the walk below always ends inside the chunk
  unsigned long long bm = __ballot(nv > 0 && incl > P);
  const bool clamp = bm == 0;
  if (clamp) bm = __ballot(nv > 0 && incl >= total);
  const int fl = first_lane(bm);
  double cum = ex;
  int hit = -1;
  if constexpr (kReg) {
#pragma unroll
    for (int q = 0; q < R; ++q) {
      cum += wv[q];
      const double cq = q == nv - 1 ? incl : fmin(cum, incl);
      if (q < nv && hit < 0 && (clamp ? cq >= total : cq > P)) hit = j0 + q;
    }
  } else {
    for (int q = 0; q < nv; ++q) {
      cum += wt(e[j0 + q]);
      const double cq = q == nv - 1 ? incl : fmin(cum, incl);
      if (hit < 0 && (clamp ? cq >= total : cq > P)) hit = j0 + q;
    }
  }
  return __builtin_amdgcn_readlane(hit, fl);
}

// Filter-level bookkeeping of the outer resampling (one thread per filter).
static __device__ void res_finish(const StepArgs& a, int f, int t, int N, const ResResult& r) {
  a.fstat[4 * f + 0] = r.deg ? 0.0 : (double)r.m;
  a.fstat[4 * f + 1] = r.total;
  a.fstat[4 * f + 2] = r.sumsq;
  a.fstat[4 * f + 3] = r.deg ? 1.0 : 0.0;
  a.ess[f] = (float)(r.total * r.total / r.sumsq);
  const double dl = r.deg ? -INFINITY : (double)r.m + log(r.total) - log((double)N);
  a.dlogz[f] = dl;
  a.loglik[f] += dl;
  uint32_t fl = r.deg ? (uint32_t)F_DEGENERATE_OUTER : 0u;
  const float* yp = a.Y + (long long)(t - 1) * a.y_tstride + (long long)f * a.dy;
  bool nonf = false;
#pragma unroll 8
  for (int q = 0; q < a.dy; ++q) nonf |= !finitef(yp[q]);
  if (nonf) fl |= F_NONFINITE;
  if (fl) atomicOr(&a.flags[f], fl);
}

// Group statistics; with advance_time, group 0's workgroup also advances the
// filter's time and flips its state copy (no other workgroup of this launch
// reads them).  In the learned step's second pass (fb set) a filter that
// kept its learned proposals keeps the statistics of the first pass.
static __global__ __launch_bounds__(kBlock) void k_res_stats(StepArgs a, const int2* rgroups, int advance_time) {
  __shared__ ResScratch sh;
  const int2 rg = rgroups[blockIdx.x];
  const int4 gi = a.ginfo[blockIdx.x];  // static: the filter's offsets and groups
  const int f = rg.x;
  const int oo = gi.x, N = gi.y, rb = gi.z;
  const int i = rg.y * kResGroup + threadIdx.x;
  // the group's log-weight (clamped index, masked below) and the filter's
  // values in one memory round (a load under a branch would wait inside it)
  const float lw = a.logw[oo + min(i, N - 1)];
  const int ac = a.act[f];
  const int fbv = a.fb != nullptr ? a.fb[f] : 1;
  const int tc = a.tcur[f], cu = a.cur[f];
  asm volatile("" ::"v"(ac), "v"(fbv), "v"(tc), "v"(cu));
  if (!ac) return;
  if (fbv == 0) {
    if (advance_time && rg.y == 0 && threadIdx.x == 0) {
      a.tcur[f] = tc + 1;
      a.cur[f] = (unsigned char)(cu ^ 1);
    }
    return;
  }
  float mg;
  double sg, qg;
  res_group_stat_lw(lw, i < N, mg, sg, qg, sh);
  const float v = i < N ? lw : 0.f;
  const int nonf = __syncthreads_or((!finitef(v) && !(v == -INFINITY)) ? 1 : 0);
  if (threadIdx.x == 0) {
    double* gs = a.gstat + 4LL * (rb + rg.y);
    gs[0] = (double)mg;
    gs[1] = sg;
    gs[2] = qg;
    if (nonf) atomicOr(&a.flags[f], (uint32_t)F_NONFINITE);
    if (advance_time && rg.y == 0) {
      a.tcur[f] = tc + 1;
      a.cur[f] = (unsigned char)(cu ^ 1);
    }
  }
}

// Outer ancestors of 256 new particles per workgroup (the grid of k_res_stats,
// after the time advance), by the group-statistics rule of resolve_points;
// group 0 also records the filter's ESS, evidence and flags.  In a learned
// step whose proposals were accepted (fb[f] == 0) the workgroup also
// commits the resampled particles: slot indirection, x, and the per-particle
// moments gathered from the learned pass.
// Learned step with accepted proposals (fb[f] == 0): outer ancestors of 256
// new particles per workgroup b (the grid of k_res_stats) by the
// group-statistics rule of resolve_points, and the commit of the resampled
// particles: the learned pass propagated particle i's cloud into slot i of
// the new copy, so particle k refers to its ancestor's slot; x and the
// per-particle moments are gathered (all loads first).  Group 0 records the
// filter's ESS, evidence and flags.  Filters that fell back are skipped
// (their new-cloud tiles resolve their own ancestors).
template <int DX, int DZ>
__device__ void commit_group(const StepArgs& a, int b) {
  __shared__ ResScratch rsh;
  __shared__ int res[kBlock];
  const int2 rg = a.rgroups[b];
  const int f = rg.x;
  // the filter's values in one memory round (a load under a branch would
  // wait inside it)
  const int ac = a.act[f], fbv = a.fb[f], N = a.fN[f], oo = a.ooff[f], t = a.tcur[f], cu = a.cur[f];
  const int rb = a.finfo[f].rg_base, G = a.finfo[f].ngroup;
  asm volatile("" ::"v"(ac), "v"(fbv), "v"(N), "v"(oo), "v"(t), "v"(cu), "v"(rb), "v"(G));
  if (!ac || fbv) return;
  const int k0 = rg.y * kResGroup;
  const int np = min(kResGroup, N - k0);
  const Key key = make_key(a.seed, (uint32_t)f);
  const double u = uniform53(key, (uint32_t)t, 0u, P_OUTER_U);
  const ResResult rr = resolve_points(LogSrc{a.logw + oo}, N, N, u, k0, np, a.gstat + 4LL * rb, G, res, rsh,
                                      rg.y == 0);
  if (rg.y == 0 && threadIdx.x == 0) res_finish(a, f, t, N, rr);
  const int th = threadIdx.x;
  const int dst = copy_of((unsigned char)cu);
  if (th < np) {
    const long long gk = oo + k0 + th, gp = oo + res[th];
    float xv[DX], kv[DZ], mv[2 * DZ];
#pragma unroll
    for (int d = 0; d < DX; ++d) xv[d] = a.xtmp[(long long)d * a.NT + gp];
#pragma unroll
    for (int d = 0; d < DZ; ++d) kv[d] = a.kpart_tmp[gp * DZ + d];
#pragma unroll
    for (int d = 0; d < 2 * DZ; ++d) mv[d] = a.mom_tmp[gp * 2 * DZ + d];
    a.anc[gk] = res[th];
    a.ind[dst][gk] = res[th];
#pragma unroll
    for (int d = 0; d < DX; ++d) a.x[dst][(long long)d * a.NT + gk] = xv[d];
#pragma unroll
    for (int d = 0; d < DZ; ++d) a.kpart[gk * DZ + d] = kv[d];
    if (a.mom) {
#pragma unroll
      for (int d = 0; d < 2 * DZ; ++d) a.mom[gk * 2 * DZ + d] = mv[d];
    }
    if (k0 == 0 && th == 0) a.cur[f] = (unsigned char)(cu & ~(2 << dst));
  }
  if (rg.y == 0 && th == 0) {
    const uint32_t lf = a.lflags[f];
    if (lf) atomicOr(&a.flags[f], lf);
    a.lflags[f] = 0u;
  }
}

// ---------------------------------------------------------------- estimates
// One workgroup per filter, FP64 sums in a fixed order (strided per thread,
// then DPP and the wave results in order), so results are reproducible.
// Used by the plain DPF (the look-ahead steps end with k_post):
//   plain:      xhat = sum_i Wbar_i xt_i, zhat = sum_i Wbar_i sum_j qbar z
//               over the proposals weighted at this step (previous copy)
template <int DX, int DZ>
constexpr int fin_block() { return DX + DZ > 16 ? 256 : 1024; }

template <int DX, int DZ, bool PLAIN>
static __global__ __launch_bounds__((fin_block<DX, DZ>())) void k_finalize(StepArgs a) {
  constexpr int NV = DX + DZ;
  constexpr int BS = fin_block<DX, DZ>();
  __shared__ double red[NV][BS / kWave];
  const int f = blockIdx.x;
  if (!a.act[f]) return;
  const int N = a.fN[f];
  const int oo = a.ooff[f];
  const int t = a.tcur[f];
  const float* xs = a.x[PLAIN ? copy_of(a.cur[f]) ^ 1 : copy_of(a.cur[f])];
  double mx = 0.0, tot = 1.0;
  bool deg = false;
  if (PLAIN) {
    mx = a.fstat[4 * f + 0];
    tot = a.fstat[4 * f + 1];
    deg = a.fstat[4 * f + 3] != 0.0;
  }
  double acc[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) acc[q] = 0.0;
  // unrolled so that the loads of several particles are in flight together
  // (same summation order as the plain loop)
#pragma unroll 4
  for (int i = threadIdx.x; i < N; i += BS) {
    double w;
    if (PLAIN) {
      const float lw = a.logw[oo + i];
      w = deg ? 1.0 / N : (finitef(lw) ? (double)fast_exp(lw - (float)mx) / tot : 0.0);
    } else {
      w = 1.0 / N;
    }
    for (int d = 0; d < DX; ++d) acc[d] += w * (double)xs[(long long)d * a.NT + oo + i];
    for (int d = 0; d < DZ; ++d) acc[DX + d] += w * (double)a.kpart[(long long)(oo + i) * DZ + d];
  }
  for (int q = 0; q < NV; ++q) {
    const double v = seg_reduce_wave<OpAdd, kWave>(acc[q]);
    if ((threadIdx.x & (kWave - 1)) == 0) red[q][threadIdx.x / kWave] = v;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < NV; q += BS) {
    double v = 0.0;
    for (int w = 0; w < BS / kWave; ++w) v += red[q][w];
    if (q < DX) {
      a.est_x[f * DX + q] = (float)v;
      if (a.trace_x) a.trace_x[((long long)(t - 1) * a.n_filters + f) * DX + q] = (float)v;
    } else {
      a.est_z[f * DZ + q - DX] = (float)v;
      if (a.trace_z) a.trace_z[((long long)(t - 1) * a.n_filters + f) * DZ + q - DX] = (float)v;
    }
  }
}

// ------------------------------------------------------- look-ahead step end
// One workgroup per resampling group of every filter (the grid of
// k_res_stats):
//  * the estimates of the step just taken, xhat = mean_k x_t^(k) and zhat =
//    mean_k sum_j qbar z (eq:qbar), as per-group FP64 partial sums (wave
//    sums, then the four waves in order) that the filter's last workgroup
//    adds up in group order -- the same order in every path, so results
//    do not depend on how the steps were launched;
//  * in a look-ahead run (next = 1), whose new-cloud kernel has already
//    computed the next step's outer log-weights: what k_res_stats does
//    before an ordinary step -- the group statistics of those weights,
//    the non-finite check, and (last workgroup) the time advance -- plus
//    the filter's activity for the next step.
// The last workgroup of a filter is found with a counter it resets.
// YH: also the predicted observation yhat = (1/N) sum_i yp_i (one more
// partial sum per group).
template <int DX, int DZ, bool YH>
__device__ __forceinline__ void post_finish(const StepArgs& a, int f, int rb, int G, int t, unsigned char cb,
                                            int next, bool act_next, int nthreads);

template <int DX, int DZ, bool YH>
static __global__ __launch_bounds__(kBlock) void k_post(StepArgs a, const int2* rgroups, int next, int split) {
  constexpr int NV = DX + DZ + (YH ? 1 : 0);
  __shared__ ResScratch sh;
  __shared__ double part[kBlock / kWave][NV];
  __shared__ int last;
  const int2 rg = rgroups[blockIdx.x];
  const int4 gi = a.ginfo[blockIdx.x];  // static: the filter's offsets and groups
  const int f = rg.x, g = rg.y;
  const int oo = gi.x, N = gi.y, rb = gi.z, G = gi.w;
  const int i = g * kResGroup + threadIdx.x;
  // loads at a clamped index, masked afterwards (a load guarded by i < N
  // would wait inside its own branch: one memory round per value); the
  // particles' values do not depend on the filter's time, so they are
  // fetched in the same memory round as it (x from both state copies)
  const int ic = min(i, N - 1);
  float raw[NV], xo[DX];
#pragma unroll
  for (int d = 0; d < DX; ++d) {
    raw[d] = a.x[0][(long long)d * a.NT + oo + ic];
    xo[d] = a.x[1][(long long)d * a.NT + oo + ic];
  }
#pragma unroll
  for (int d = 0; d < DZ; ++d) raw[DX + d] = a.kpart[(long long)(oo + ic) * DZ + d];
  if constexpr (YH) raw[NV - 1] = a.yp[oo + ic];
  const float lwn = (next && a.logw_next != nullptr) ? a.logw_next[oo + ic] : 0.f;
  const int tf = (next && a.run_Tf != nullptr) ? a.run_Tf[f] : 0x7fffffff;
  const int act = a.act[f], t = a.tcur[f], cu = a.cur[f];  // t: the step just taken
  asm volatile("" ::"v"(tf), "v"(act), "v"(t), "v"(cu));
  if (!act) return;
  const unsigned char cb = (unsigned char)cu;
  if (copy_of(cb)) {
#pragma unroll
    for (int d = 0; d < DX; ++d) raw[d] = xo[d];
  }
  const double w = 1.0 / N;
  const bool act_next = next && t < min(tf, a.run_T);
  double v[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = i < N ? w * (double)raw[q] : 0.0;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    const double r = seg_reduce_wave<OpAdd, kWave>(v[q]);
    if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave][q] = r;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < NV; q += kBlock)
    a.gpart[(long long)(rb + g) * NV + q] = ((part[0][q] + part[1][q]) + part[2][q]) + part[3][q];
  if (act_next) {
    float mg;
    double sg, qg;
    res_group_stat_lw(lwn, i < N, mg, sg, qg, sh);
    const float lv = i < N ? lwn : 0.f;
    const int nonf = __syncthreads_or((!finitef(lv) && !(lv == -INFINITY)) ? 1 : 0);
    if (threadIdx.x == 0) {
      double* gs = a.gstat + 4LL * (rb + g);
      gs[0] = (double)mg;
      gs[1] = sg;
      gs[2] = qg;
      if (nonf) atomicOr(&a.flags[f], (uint32_t)F_NONFINITE);
    }
  }
  if (split) return;  // k_post_end finishes the filters
  __threadfence();
  if (threadIdx.x == 0) last = atomicAdd(&a.fcount[f], 1) == G - 1;
  __syncthreads();
  if (!last) return;
  __threadfence();
  if (threadIdx.x == 0) a.fcount[f] = 0;
  post_finish<DX, DZ, YH>(a, f, rb, G, t, cb, next, act_next, kBlock);
}

// Filter-level end of k_post: the estimates from the group partials (in
// group order), the next step's activity and the time advance.
template <int DX, int DZ, bool YH>
__device__ __forceinline__ void post_finish(const StepArgs& a, int f, int rb, int G, int t, unsigned char cb,
                                            int next, bool act_next, int nthreads) {
  constexpr int NV = DX + DZ + (YH ? 1 : 0);
  for (int q = threadIdx.x; q < NV; q += nthreads) {
    double e = 0.0;
    // (unrolled: the loads of several groups in flight, added in order)
#pragma unroll 16
    for (int gg = 0; gg < G; ++gg) e += a.gpart[(long long)(rb + gg) * NV + q];
    if (q < DX) {
      a.est_x[f * DX + q] = (float)e;
      if (a.trace_x) a.trace_x[((long long)(t - 1) * a.n_filters + f) * DX + q] = (float)e;
    } else if (q < DX + DZ) {
      a.est_z[f * DZ + q - DX] = (float)e;
      if (a.trace_z) a.trace_z[((long long)(t - 1) * a.n_filters + f) * DZ + q - DX] = (float)e;
    } else {
      a.est_y[f] = (float)e;
      if (a.trace_y) a.trace_y[(long long)(t - 1) * a.n_filters + f] = (float)e;
    }
  }
  if (threadIdx.x == 0 && next) {
    a.act[f] = act_next ? 1 : 0;
    if (act_next) {
      a.tcur[f] = t + 1;
      a.cur[f] = (unsigned char)(cb ^ 1);
    }
  }
}

// With many groups in a launch the cross-workgroup hand-off of k_post (a
// device-scope fence per workgroup writes back the L2 of its XCD) costs more
// than a kernel boundary: k_post runs split (groups only) and this kernel,
// one 64-thread workgroup per filter, finishes the filters.
template <int DX, int DZ, bool YH>
static __global__ __launch_bounds__(kWave) void k_post_end(StepArgs a, int next) {
  const int f = blockIdx.x;
  const int tf = (next && a.run_Tf != nullptr) ? a.run_Tf[f] : 0x7fffffff;
  const int rb = a.finfo[f].rg_base;
  asm volatile("" ::"v"(tf), "v"(rb));
  const FilterView fv = load_filter(a, f);
  if (!fv.act) return;
  const bool act_next = next && fv.t < min(tf, a.run_T);
  post_finish<DX, DZ, YH>(a, f, rb, fv.ngroup, fv.t, (unsigned char)fv.cur, next, act_next, kWave);
}

// ---------------------------------------------------------------- new cloud
// Look-ahead mode (Fig. 4 step 4): new particle k with parent p = anc[k]
//  * selects candidate c over the parent's ell by one inverse-CDF draw
//    (U53 CAND_U at (t, k, 0)) and regenerates x_t = xla^{(p,c)} from the
//    LA_X normals at (t, p, c) (eq:approx3, sampled by SIR);
//  * conditions the parent's cloud on x_t, kappa_j = lam_pj + log p(x_t |
//    x_p, z_pj) (eq:qnobar), resamples it systematically (INNER_U);
//  * propagates z_t^{(k,j)} = f^z(x_p, x_t, z_{p,b_j}) (NEW_Z at (t, k, j));
//  * applies eq:qbar: lam_t = log p(y_t | x_t, z_t) - logsumexp_j.
// Plain mode (Fig. 2 steps 4-7): a_k ~ Cat(qbar_p) (DPF_ANC_U), a fresh
// x_{t+1} from the a_k-th component (DPF_X at (t, k, 0)), kappa = ell_pj +
// log p(x_{t+1} | x_p, z_pj), systematic inner resampling, DPF_Z normals;
// no measurement update (that happens at the next step).
template <class Mdl, int SEG, int JPT, bool PLAIN>
__device__ __forceinline__ void newcloud_tile(const StepArgs& a, int ti) {
  constexpr int DX = Mdl::DX, DZ = Mdl::DZ, DY = Mdl::DY;
  constexpr int NSEG = kBlock / SEG;
  constexpr bool kKeepZ = JPT * DZ <= 64;  // new z stays in registers for the partial sums
  // Wide z: the propagation takes one inner particle at a time (its gathered,
  // noise and new z arrays alone fill most of the registers), passing each
  // one's likelihoods to the later loops through LDS.
  constexpr bool kRoll = DZ >= 32 && JPT > 1;
  constexpr bool kStream = Mdl::kStreamZ;
  __shared__ SegScratch sh;
  __shared__ double cdf[NSEG][SEG * JPT];
  __shared__ float roll_sh[kRoll ? 2 * JPT : 1][kRoll ? kBlock : 1];
  __shared__ float xs_sh[NSEG][DX];
  __shared__ int csel[NSEG];
  __shared__ float vred[kBlock / kWave][2 * DZ];
  __shared__ int anc_sh[NSEG];
  __shared__ ResScratch rsh;

  const int4 tile = a.tiles[ti];
  const int f = tile.x;
  // group statistics for the wave-level ancestor draw, lane l: group l of
  // the filter (fetched with the filter's values; the array is padded)
  double gst[3] = {0.0, 0.0, 0.0};
  if constexpr (SEG >= kWave) {
    const double* gp = a.gstat + 4LL * (tile.w + (threadIdx.x & (kWave - 1)));
    gst[0] = gp[0];
    gst[1] = gp[1];
    gst[2] = gp[2];
  }
  // the next step's horizon (look-ahead run)
  const int tf_next = (!PLAIN && a.ell_next != nullptr && a.run_Tf != nullptr) ? a.run_Tf[f] : 0x7fffffff;
  const FilterView fv = load_filter(a, f);
  if (!fv.act) return;
  // learned step with accepted proposals: committed by commit_group
  if (!PLAIN && fv.fb == 0) return;
  // look-ahead run: this kernel also computes the next step's weights (Fig. 4
  // steps 1-2 at t + 1) for the filters that take it; y_{t+1} fetched early
  const bool fuse = !PLAIN && a.ell_next != nullptr && fv.t < min(tf_next, a.run_T);
  float yn[DY];
  if (!PLAIN && a.ell_next != nullptr) load_y<Mdl>(a, f, min(fv.t, a.run_T - 1) + 1, yn);
  const int N = fv.N, M = fv.M;
  const int s = threadIdx.x / SEG;
  const int ls = threadIdx.x % SEG;
  const int k = tile.y + s;
  const bool vk = k < N;
  const int oo = fv.oo;
  const long long io = fv.io;
  const int t = fv.t;  // already advanced (0 at initialisation)
  const unsigned char cb = (unsigned char)fv.cur;
  const int dst = copy_of(cb), src = dst ^ 1;
  const Key key = make_key(a.seed, (uint32_t)f);

  // With a wave or more per outer particle, the ancestor and the candidate
  // are single draws done by the segment's first wave with wave-wide scans.
  // The NEW_Z / DPF_Z normals of the inner particles do not depend on them:
  // the segment's other waves draw theirs meanwhile.
  constexpr bool kWaveDraw = SEG >= kWave;
  constexpr bool kEarly = SEG > kWave && JPT * DZ <= 16;
  static_assert(!(kEarly && kStream), "a streamed model draws its noise in the propagation");
  float nue[kEarly ? JPT : 1][DZ];
  // One wave per outer particle: the parent's kappa inputs (lam, or ell in
  // plain mode, and z when p(x'|x, z) depends on z) are fetched together
  // with its ell row for the candidate draw, in the same memory round.
  constexpr bool kPre = SEG == kWave;
  constexpr bool kPreZ = kPre && Mdl::kXdepZ;
  constexpr bool kXZ = Mdl::kXdepZ;
  constexpr int NPX = npx<Mdl>();
  float kpre[kPre ? JPT : 1];
  float zpre[kPreZ ? JPT : 1][kPreZ ? DZ : 1];
#pragma unroll
  for (int r = 0; r < (kPre ? JPT : 1); ++r) {
    kpre[r] = 0.f;
#pragma unroll
    for (int d = 0; d < (kPreZ ? DZ : 1); ++d) zpre[r][d] = 0.f;
  }
  int p, c, pc;
  bool deg1;
  float xp[DX], xn[DX];
  if constexpr (kWaveDraw) {
    // ---- 0-2. ancestor, candidate and new x by the segment's first wave --
    __shared__ int pc_sh[NSEG][2];
    __shared__ float xw_sh[NSEG][DX];
    __shared__ int d1_sh[NSEG];
    const int G = fv.ngroup;
    const bool resolve = a.advance && !a.anc_ready;
    const bool blk = resolve && G > kWave;  // many groups: the whole workgroup resolves
    if (blk) {
      const double u = uniform53(key, (uint32_t)t, 0u, P_OUTER_U);
      const ResResult rr = resolve_points(LogSrc{a.logw + oo}, N, N, u, tile.y, min(NSEG, N - tile.y),
                                          a.gstat + 4LL * a.finfo[f].rg_base, G, anc_sh, rsh, tile.z == 0);
      if (tile.z == 0 && threadIdx.x == 0) res_finish(a, f, t, N, rr);
    }
    int pw = 0, cw = 0, pcw = 0;
    bool d1 = false;
    float xpw[DX], xw[DX];
#pragma unroll
    for (int d = 0; d < DX; ++d) xpw[d] = xw[d] = 0.f;
    if (ls < kWave && vk) {
      if (blk) {
        pw = anc_sh[s];
      } else if (resolve) {
        ResResult rr;
        const double u = uniform53(key, (uint32_t)t, 0u, P_OUTER_U);
        const bool first = tile.z == 0 && s == 0;
        pw = resolve_point_w0(LogSrc{a.logw + oo}, N, N, u, k, gst, G, first, rr);
        if (first && ls == 0) res_finish(a, f, t, N, rr);
      } else {
        pw = a.advance ? a.anc[oo + k] : k;  // identity at initialisation
      }
      // the parent's slot and x do not depend on the candidate: fetched first
      pcw = (PLAIN || ident_slots(cb, src)) ? pw : a.ind[src][oo + pw];
#pragma unroll
      for (int d = 0; d < DX; ++d) xpw[d] = a.x[src][(long long)d * a.NT + oo + pw];
      const float* zpw = a.z[src] + (io + (long long)pcw * M) * DZ;
      if constexpr (kPre) {
        const float* kr = PLAIN ? a.ell + io + (long long)pw * M : a.lam[src] + io + (long long)pcw * M;
#pragma unroll
        for (int r = 0; r < JPT; ++r) {
          const int j = ls + r * SEG;
          if (j < M) {
            kpre[r] = kr[j];
            if constexpr (kPreZ) {
#pragma unroll
              for (int d = 0; d < DZ; ++d) zpre[kPreZ ? r : 0][kPreZ ? d : 0] = zpw[d * M + j];
            }
          }
        }
      }
      // candidate (look-ahead) / inner ancestor (plain) over the parent's ell
      const double uc = uniform53(key, (uint32_t)t, (uint32_t)k, PLAIN ? P_DPF_ANC_U : P_CAND_U);
      cw = select_w0<(SEG * JPT + kWave - 1) / kWave>(a.ell + io + (long long)pw * M, M, uc, d1);
      // every lane of the wave computes the new x (same counters)
      float zc[DZ], nu[DX];
      if constexpr (kPreZ) {
        // z of the candidate: held by lane cw % 64 in its slot cw / 64
        const int rr = cw / SEG;
#pragma unroll
        for (int d = 0; d < DZ; ++d) {
          float v = zpre[0][kPreZ ? d : 0];
#pragma unroll
          for (int r = 1; r < JPT; ++r)
            if (rr == r) v = zpre[kPreZ ? r : 0][kPreZ ? d : 0];
          zc[d] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), cw % SEG));
        }
      } else {
#pragma unroll
        for (int d = 0; d < DZ; ++d) zc[d] = zpw[d * M + cw];
      }
      if (PLAIN)
        normals<DX>(key, (uint32_t)t, (uint32_t)k, 0u, P_DPF_X, nu);
      else
        normals<DX>(key, (uint32_t)t, (uint32_t)pw, (uint32_t)cw, P_LA_X, nu);
      Mdl::fx(as_prm(a.prm), xpw, zc, nu, PLAIN ? t : t - 1, xw);
      if (ls == 0) {
        if (!a.anc_ready) a.anc[oo + k] = pw;
        a.sel[oo + k] = cw;
#pragma unroll
        for (int d = 0; d < DX; ++d) a.x[dst][(long long)d * a.NT + oo + k] = xw[d];
      }
    }
    if constexpr (SEG == kWave) {
      p = pw;
      c = cw;
      pc = pcw;
      deg1 = d1;
#pragma unroll
      for (int d = 0; d < DX; ++d) {
        xn[d] = xw[d];
        xp[d] = xpw[d];
      }
    } else {
      if (ls == 0) {
#pragma unroll
        for (int d = 0; d < DX; ++d) xw_sh[s][d] = xw[d];
        pc_sh[s][0] = pw;
        pc_sh[s][1] = cw;
        d1_sh[s] = d1 ? 1 : 0;
      }
      if constexpr (kEarly) {
#pragma unroll
        for (int r = 0; r < JPT; ++r) {
          const int jj = ls + r * SEG;
          if (jj < M) normals<DZ>(key, (uint32_t)t, (uint32_t)k, (uint32_t)jj, PLAIN ? P_DPF_Z : P_NEW_Z, nue[r]);
        }
      }
      __syncthreads();
      p = pc_sh[s][0];
      c = pc_sh[s][1];
      deg1 = d1_sh[s] != 0;
#pragma unroll
      for (int d = 0; d < DX; ++d) xn[d] = xw_sh[s][d];
      pc = (PLAIN || ident_slots(cb, src)) ? p : a.ind[src][oo + p];
#pragma unroll
      for (int d = 0; d < DX; ++d) xp[d] = a.x[src][(long long)d * a.NT + oo + p];
    }
  } else {
  // ---- 0. outer ancestors of this tile's new particles -------------------
  // (resolved here, also for the learned step's fallback filters)
  if (a.advance && !a.anc_ready) {
    const int np = min(NSEG, N - tile.y);
    const int G = a.finfo[f].ngroup;
    const double u = uniform53(key, (uint32_t)t, 0u, P_OUTER_U);
    const ResResult rr = resolve_points(LogSrc{a.logw + oo}, N, N, u, tile.y, np,
                                        a.gstat + 4LL * a.finfo[f].rg_base, G, anc_sh, rsh, tile.z == 0);
    if (tile.z == 0 && threadIdx.x == 0) res_finish(a, f, t, N, rr);
  } else if (threadIdx.x < NSEG) {
    const int kk = tile.y + threadIdx.x;
    anc_sh[threadIdx.x] = a.advance ? (kk < N ? a.anc[oo + kk] : 0) : kk;  // identity at initialisation
  }
  __syncthreads();
  p = vk ? anc_sh[s] : 0;
  if (vk && ls == 0 && !a.anc_ready) a.anc[oo + k] = p;
  pc = (PLAIN || ident_slots(cb, src)) ? p : a.ind[src][oo + p];
#pragma unroll
  for (int d = 0; d < DX; ++d) xp[d] = a.x[src][(long long)d * a.NT + oo + p];
  const float* zp0 = a.z[src] + (io + (long long)pc * M) * DZ;
  const float* ep = a.ell + io + (long long)p * M;

  // ---- 1. selection over the parent's ell (candidate / ancestor) --------
  float ev[JPT];
  float mloc = -INFINITY;
#pragma unroll
  for (int r = 0; r < JPT; ++r) {
    const int j = ls + r * SEG;
    ev[r] = (vk && j < M) ? ep[j] : -INFINITY;
    if (finitef(ev[r])) mloc = fmaxf(mloc, ev[r]);
  }
  const float m1 = seg_max<SEG>(mloc, sh);
  deg1 = !(m1 > -INFINITY);
  double carry = 0.0;
#pragma unroll
  for (int r = 0; r < JPT; ++r) {
    const int j = ls + r * SEG;
    double w = 0.0;
    if (j < M) w = deg1 ? 1.0 : (finitef(ev[r]) ? (double)fast_exp(ev[r] - m1) : 0.0);
    double tot;
    const double c = seg_scan_incl<SEG>(w, sh, tot);
    cdf[s][r * SEG + ls] = carry + c;
    carry += tot;
  }
  __syncthreads();
  if (ls == 0) {
    const double u = uniform53(key, (uint32_t)t, (uint32_t)k, PLAIN ? P_DPF_ANC_U : P_CAND_U);
    csel[s] = vk ? cdf_search(cdf[s], M, sys_point(0, u, cdf[s][M - 1], 1)) : 0;
    if (vk) a.sel[oo + k] = csel[s];
  }
  __syncthreads();
  c = csel[s];

  // ---- 2. the new outer particle ----------------------------------------
  if (ls == 0) {
    float zc[DZ], nu[DX];
#pragma unroll
    for (int d = 0; d < DZ; ++d) zc[d] = zp0[d * M + c];
    if (PLAIN)
      normals<DX>(key, (uint32_t)t, (uint32_t)k, 0u, P_DPF_X, nu);
    else
      normals<DX>(key, (uint32_t)t, (uint32_t)p, (uint32_t)c, P_LA_X, nu);
    float xw[DX];
    Mdl::fx(as_prm(a.prm), xp, zc, nu, PLAIN ? t : t - 1, xw);
#pragma unroll
    for (int d = 0; d < DX; ++d) xs_sh[s][d] = xw[d];
    if (vk) {
#pragma unroll
      for (int d = 0; d < DX; ++d) a.x[dst][(long long)d * a.NT + oo + k] = xw[d];
    }
  }
  __syncthreads();
#pragma unroll
  for (int d = 0; d < DX; ++d) xn[d] = xs_sh[s][d];

  }
  // the new clouds are written in slot order: the slots of copy dst become
  // the identity
  if (!PLAIN && tile.z == 0 && threadIdx.x == 0 && !ident_slots(cb, dst))
    a.cur[f] = (unsigned char)(cb | (2 << dst));
  const float* zp = a.z[src] + (io + (long long)pc * M) * DZ;
  const float* ep = a.ell + io + (long long)p * M;
  (void)c;

  // ---- 3. x-conditioned inner weights and local systematic resampling ---
  const float* lp = a.lam[src] + io + (long long)pc * M;
  float ev[JPT];
  float mk = -INFINITY;
  float cpx[kXZ ? NPX : 1];
  if constexpr (kXZ) Mdl::px_pre(as_prm(a.prm), xn, xp, PLAIN ? t : t - 1, cpx);
#pragma unroll
  for (int r = 0; r < JPT; ++r) {
    const int j = ls + r * SEG;
    if (vk && j < M) {
      float kap = kPre ? kpre[kPre ? r : 0] : (PLAIN ? ep[j] : lp[j]);
      if constexpr (kXZ) {
        float zj[DZ];
#pragma unroll
        for (int d = 0; d < DZ; ++d) zj[d] = kPreZ ? zpre[kPreZ ? r : 0][kPreZ ? d : 0] : zp[d * M + j];
        kap += Mdl::logpx_post(as_prm(a.prm), cpx, zj);
      }
      ev[r] = kap;
      if (finitef(kap)) mk = fmaxf(mk, kap);
    } else {
      ev[r] = -INFINITY;
    }
  }
  const float m2 = seg_max<SEG>(mk, sh);
  const bool deg2 = !(m2 > -INFINITY);
  double carry = 0.0;
#pragma unroll
  for (int r = 0; r < JPT; ++r) {
    const int j = ls + r * SEG;
    double w = 0.0;
    if (j < M) w = deg2 ? 1.0 : (finitef(ev[r]) ? (double)fast_exp(ev[r] - m2) : 0.0);
    double tot;
    const double cc = seg_scan_incl<SEG>(w, sh, tot);
    cdf[s][r * SEG + ls] = carry + cc;
    carry += tot;
  }
  seg_lds_sync<SEG>();
  const double u_in = uniform53(key, (uint32_t)t, (uint32_t)k, P_INNER_U);
  const double tot2 = cdf[s][M - 1];

  // ---- 4. gather + propagate (+ measurement update in look-ahead mode) ---
  float pre[Mdl::NPRE];
  // (plain: t is the step just taken and the proposal is for t + 1)
  fz_pre_seg<Mdl, SEG>(as_prm(a.prm), xp, xn, PLAIN ? t : t - 1, pre);
  float y[DY], r0[DY];
  if (!PLAIN) {
    load_y<Mdl>(a, f, t, y);
    Mdl::obs_pre(as_prm(a.prm), y, xn, r0);
  }
  float* zdst = a.z[dst] + (io + (long long)k * M) * DZ;
  float llv[JPT], gn[JPT];
  float zkeep[kKeepZ ? JPT : 1][DZ];
  // predicted observation of the next step (fused run, when requested)
  constexpr bool kH = !PLAIN && has_yhat<Mdl>();
  const bool want_h = kH && fuse && a.yp_next != nullptr;
  float hn[kH ? JPT : 1];
  Lse acc;
  // wide z: the new z of every lane of the wave goes through the matrix-core
  // residual together (lanes without a particle carry zeros)
  float ca[kStream ? Mdl::DZ / 2 : 1];
  if constexpr (kStream) WaveProj<Mdl>::load_a(as_prm(a.prm), ca);
#pragma unroll kRoll ? 1 : JPT
  for (int r = 0; r < JPT; ++r) {
    const int jj = ls + r * SEG;
    float lv = -INFINITY, gv = 0.f;
    if constexpr (kStream) {
      const bool on = vk && jj < M;
      const int b = on ? cdf_search(cdf[s], M, sys_point(jj, u_in, tot2, M)) : 0;
      float zg[DZ], zn[DZ];
#pragma unroll
      for (int d = 0; d < DZ; ++d) zg[d] = on ? zp[d * M + b] : 0.f;
      const Prm P = as_prm(a.prm);
      WaveProj<Mdl> pj;
      pj.start();
      normal_pairs<0, DZ, false>(key, (uint32_t)t, (uint32_t)k, (uint32_t)jj, PLAIN ? P_DPF_Z : P_NEW_Z, 0.f,
                                 [&](int d, float n0, float n1) {
                                   zn[d] = Mdl::fz_post_k(P, pre[d], zg, n0, d);
                                   zn[d + 1] = Mdl::fz_post_k(P, pre[d + 1], zg, n1, d + 1);
                                   if (on) {
                                     zdst[d * M + jj] = zn[d];
                                     zdst[(d + 1) * M + jj] = zn[d + 1];
                                   }
                                   if (!PLAIN) pj.add(ca[d / 2], zn[d], zn[d + 1]);
                                 });
      if constexpr (kKeepZ) {
#pragma unroll
        for (int d = 0; d < DZ; ++d) zkeep[kKeepZ ? r : 0][d] = zn[d];
      }
      if (!PLAIN) {
        const float l0 = pj.logpy(P, y_row<Mdl>(a, f, t));
        // the next step's look-ahead likelihood of these new inner particles
        const float g0 = fuse ? la_logpy_wave<Mdl>(a, key, t + 1, k, jj, xn, zn,
                                                   y_row<Mdl>(a, f, min(fv.t, a.run_T - 1) + 1), ca)
                              : 0.f;
        if (on) {
          lv = l0;
          gv = g0;
          acc.add(lv);
        }
      }
    } else if (vk && jj < M) {
      const int b = cdf_search(cdf[s], M, sys_point(jj, u_in, tot2, M));
      float zg[DZ], zn[DZ], nu[DZ];
#pragma unroll
      for (int d = 0; d < DZ; ++d) zg[d] = zp[d * M + b];
      if constexpr (kEarly) {
#pragma unroll
        for (int d = 0; d < DZ; ++d) nu[d] = nue[kEarly ? r : 0][d];
      } else {
        normals<DZ>(key, (uint32_t)t, (uint32_t)k, (uint32_t)jj, PLAIN ? P_DPF_Z : P_NEW_Z, nu);
      }
      Mdl::fz_post(as_prm(a.prm), pre, zg, nu, zn);
#pragma unroll
      for (int d = 0; d < DZ; ++d) zdst[d * M + jj] = zn[d];
      if (!PLAIN) lv = Mdl::logpy_post(as_prm(a.prm), r0, zn);
      if constexpr (kKeepZ) {
#pragma unroll
        for (int d = 0; d < DZ; ++d) zkeep[kKeepZ ? r : 0][d] = zn[d];
      }
      if (!PLAIN) {
        acc.add(lv);
        // the next step's look-ahead likelihood of this new inner particle
        // (ALU work that overlaps the gathers of the others)
        if (want_h) {
          float h[1];
          gv = la_logpy<Mdl, kH>(a, key, t + 1, k, jj, xn, zn, yn, h);
          hn[kH ? r : 0] = h[0];
        } else if (fuse) {
          gv = la_logpy<Mdl>(a, key, t + 1, k, jj, xn, zn, yn);
        }
      }
    }
    if constexpr (kRoll) {
      roll_sh[2 * r][threadIdx.x] = lv;
      roll_sh[2 * r + 1][threadIdx.x] = gv;
    } else {
      llv[r] = lv;
      gn[r] = gv;
    }
  }
  if constexpr (kRoll) {
    // (each thread reads back its own slots)
#pragma unroll
    for (int r = 0; r < JPT; ++r) {
      llv[r] = roll_sh[2 * r][threadIdx.x];
      gn[r] = roll_sh[2 * r + 1][threadIdx.x];
    }
  }
  uint32_t fl = (deg1 || deg2) ? (uint32_t)F_DEGENERATE_INNER : 0u;
  if (!PLAIN) {
    const float lse = seg_lse<SEG>(acc, sh);
    const bool deg3 = !(lse > -INFINITY);
    if (deg3) fl |= F_DEGENERATE_INNER;
    float* ldst = a.lam[dst] + io + (long long)k * M;
    constexpr int NP = has_moments<Mdl>() ? 2 * DZ : DZ;
    const bool want_mom = has_moments<Mdl>() && a.mom != nullptr;
    float part[NP];
    float lamv[JPT];
#pragma unroll
    for (int d = 0; d < NP; ++d) part[d] = 0.f;
#pragma unroll
    for (int r = 0; r < JPT; ++r) {
      const int jj = ls + r * SEG;
      lamv[r] = 0.f;
      if (vk && jj < M) {
        const float lam = deg3 ? -fast_log((float)M) : (finitef(llv[r]) ? llv[r] - lse : -INFINITY);
        lamv[r] = lam;
        ldst[jj] = lam;
        const float q = deg3 ? 1.0f / (float)M : (finitef(llv[r]) ? fast_exp(lam) : 0.f);
#pragma unroll
        for (int d = 0; d < DZ; ++d) {
          const float zv = kKeepZ ? zkeep[kKeepZ ? r : 0][d] : zdst[d * M + jj];
          part[d] += q * zv;
          if constexpr (NP == 2 * DZ) part[DZ + d] += want_mom ? q * zv * zv : 0.f;
        }
      }
    }
    float* kp = a.kpart + (long long)(oo + k) * DZ;
    if constexpr (NP <= 16) {
      // transpose reduction: each owning lane stores its slot
      int slot;
      if (want_mom) {
        const float tot = seg_sum_vec_t<SEG, NP>(part, reinterpret_cast<float(*)[NP]>(&vred[0][0]), slot);
        const float mean = seg_vec_fetch<SEG, NP>(tot, slot >= DZ ? slot - DZ : -1);
        if (vk && slot >= 0) {
          float* mp = a.mom + (long long)(oo + k) * 2 * DZ;
          if (slot < DZ) {
            kp[slot] = tot;
            mp[slot] = tot;
          } else {
            mp[slot] = fmaxf(tot - mean * mean, 0.f);
          }
        }
      } else {
        const float tot = seg_sum_vec_t<SEG, DZ>(part, reinterpret_cast<float(*)[DZ]>(&vred[0][0]), slot);
        if (vk && slot >= 0) kp[slot] = tot;
      }
    } else {
      seg_sum_vec<SEG, DZ>(part, reinterpret_cast<float(*)[DZ]>(&vred[0][0]));
      if (vk && ls == 0) {
#pragma unroll
        for (int d = 0; d < DZ; ++d) kp[d] = part[d];
      }
    }
    // ---- 5. look-ahead run: the next step's weights ell = lam + g, in the
    // weights kernel's lane layout and summation order
    if (fuse) {
      float* en = a.ell_next + io + (long long)(vk ? k : 0) * M;
      Lse acc2;
      float hv = 0.f;
#pragma unroll
      for (int r = 0; r < JPT; ++r) {
        const int jj = ls + r * SEG;
        if (vk && jj < M) {
          const float e = la_ell(lamv[r], gn[r]);
          en[jj] = e;
          acc2.add(e);
          if (want_h) hv += fast_exp(lamv[r]) * hn[kH ? r : 0];
        }
      }
      const float lw = seg_lse<SEG>(acc2, sh);
      if (vk && ls == 0) a.logw_next[oo + k] = lw;
      if (want_h) {
        const float hs = seg_sum<SEG>(hv, sh);
        if (vk && ls == 0) a.yp_next[oo + k] = hs;
      }
    }
  }
  if (vk && ls == 0 && fl) atomicOr(&a.flags[f], fl);
}

// Workgroups are dealt to the eight XCDs in turn (workgroup b to XCD b % 8).
// The tile of workgroup b when each XCD instead takes one contiguous run of
// the n tiles: a bijection of [0, n).
__device__ __forceinline__ int xcd_contiguous_tile(int b, int n) {
  constexpr int kXcd = 8;
  const int q = n / kXcd, r = n % kXcd, x = b % kXcd;
  return x * q + min(x, r) + b / kXcd;
}

// With the wide inner state the children of one parent (neighbouring tiles
// after the ordered resampling) run on one XCD and read the parent's cloud
// through one L2.
template <class Mdl, int SEG, int JPT, bool PLAIN>
static __global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(min_waves<Mdl>()))) void k_newcloud(StepArgs a) {
  const int ti = Mdl::kStreamZ ? xcd_contiguous_tile((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x;
  newcloud_tile<Mdl, SEG, JPT, PLAIN>(a, ti);
}

// Learned step: the new clouds of the filters that fell back only (smaller
// grid looping over the tiles, tiles checked at once).
template <class Mdl, int SEG, int JPT>
static __global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(min_waves<Mdl>()))) void k_newcloud_fallback(StepArgs a) {
  constexpr bool PLAIN = false;
  // the first n_commit workgroups commit the filters that kept their
  // learned proposals
  if ((int)blockIdx.x < a.n_commit) {
    commit_group<Mdl::DX, Mdl::DZ>(a, blockIdx.x);
    return;
  }
  const int bid = blockIdx.x - a.n_commit, nb = gridDim.x - a.n_commit;
  __shared__ int todo[kBlock], wcnt[kBlock / kWave];
  for (int base = bid; base < a.n_tiles; base += kBlock * nb) {
    const int mine = base + threadIdx.x * nb;
    // tile, then both of its filter's bytes in one round (clamped, masked)
    const int f = a.tiles[min(mine, a.n_tiles - 1)].x;
    const int ac = a.act[f], fbv = a.fb[f];
    const bool need = mine < a.n_tiles && ac && fbv;
    const int nt = block_compact(need, mine, todo, wcnt, nullptr);
    for (int q = 0; q < nt; ++q) {
      newcloud_tile<Mdl, SEG, JPT, PLAIN>(a, todo[q]);
      __syncthreads();
    }
  }
}

}  // namespace dpf
