// Step with a learned proposal for the outer block (the importance-sampling
// step of Fig. 2, step 1, with a trained mixture density q in place of the
// prior), falling back to the look-ahead step of Fig. 4 for every filter
// whose effective sample size drops below a set fraction of N.
//
// Launch sequence of one step (each kernel gated per filter):
//   k_mlp_fwd_state        features of every outer particle -> mixture
//                          outputs; its epilogue draws x_t ~ q (MDN_U, MDN_X
//                          at (t, i)) and log q (k_mdn_draw instead when the
//                          caller supplies the outputs)
//   k_learned_inner        condition particle i's inner cloud on x_t
//                          (eq:qnobar, eq:approx1), resample it locally
//                          (INNER_U), propagate (NEW_Z at (t, i, j)),
//                          measurement update (eq:approx2, eq:qbar), and
//                          log w_i = log p_Nz(y_t | .) + log p_Nz(x_t | .) - log q
//   k_res_stats            group statistics of log w (no time advance)
//   k_la_weights_fallback  per filter: reject when ESS < ess_frac N; the
//                          rejecting filters' look-ahead weights
//   k_res_stats            statistics (look-ahead weights, or the same
//                          learned ones again) and the time advance
//   k_newcloud_fallback    head workgroups: resample and commit the accepted
//                          filters; the rest: look-ahead new clouds of the
//                          filters that fell back
//   k_post                 estimates
// Accepted particles are not copied: particle i's new cloud is written to
// its own slot of the next state copy and the resampled particle k refers to
// slot A_k through ind (lazy resampling); x and the per-particle moments are
// gathered.
#pragma once
#include <hip/hip_runtime.h>

#include "dpf_kernels.hpp"
#include "dpf_mlp.hpp"

namespace dpf {

// Filter of global outer index g (offsets off[0..F], off[0] = 0).
__device__ __forceinline__ int filter_of_outer(const int* off, int F, int g) {
  int lo = 0, hi = F - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= g)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Draw from the mixture of output row o: component by one inverse-CDF draw
// over softmax(logits) with U53 MDN_U at (t, i), then mean + sd * normals
// (MDN_X at (t, i, 0)); returns log q of the draw.
template <int DX>
__device__ float mdn_draw(const float* o, Key key, int t, int i, float* x, int& comp) {
  using Q = Mdn<DX>;
  float lmax = -INFINITY;
#pragma unroll
  for (int c = 0; c < kMix; ++c)
    if (finitef(o[c])) lmax = fmaxf(lmax, o[c]);
  double C[kMix];
  double acc = 0.0;
#pragma unroll
  for (int c = 0; c < kMix; ++c) {
    const double w = lmax > -INFINITY ? (finitef(o[c]) ? (double)fast_exp(o[c] - lmax) : 0.0) : 1.0;
    acc += w;
    C[c] = acc;
  }
  const double u = uniform53(key, (uint32_t)t, (uint32_t)i, P_MDN_U);
  const double P = sys_point(0, u, C[kMix - 1], 1);
  // the search rule of cdf_search, unrolled so that C stays in registers
  comp = -1;
#pragma unroll
  for (int c = 0; c < kMix; ++c)
    if (comp < 0 && C[c] > P) comp = c;
#pragma unroll
  for (int c = 0; c < kMix; ++c)
    if (comp < 0 && C[c] >= C[kMix - 1]) comp = c;
  float nu[DX];
  normals<DX>(key, (uint32_t)t, (uint32_t)i, 0u, P_MDN_X, nu);
  float mu[DX], sd[DX];
#pragma unroll
  for (int d = 0; d < DX; ++d) mu[d] = sd[d] = 0.f;
#pragma unroll
  for (int c = 0; c < kMix; ++c) {
    if (c == comp) {
#pragma unroll
      for (int d = 0; d < DX; ++d) {
        mu[d] = o[Q::kMu + c * DX + d];
        sd[d] = clamp_sd(o[Q::kSd + c * DX + d]);
      }
    }
  }
#pragma unroll
  for (int d = 0; d < DX; ++d) x[d] = mu[d] + fast_exp(sd[d]) * nu[d];
  return mdn_logpdf<DX>(o, x);
}

// The proposal of outer particle g (filter f, local index i) from its
// mixture outputs o: x_t -> xtmp, log q -> logq, component -> sel.
template <int DX>
__device__ __forceinline__ void mdn_propose(const StepArgs& a, int f, int g, const float* o) {
  const int i = g - a.ooff[f];
  const int t = a.tcur[f] + 1;
  float xn[DX];
  int comp;
  const float lq = mdn_draw<DX>(o, make_key(a.seed, (uint32_t)f), t, i, xn, comp);
#pragma unroll
  for (int d = 0; d < DX; ++d) a.xtmp[(long long)d * a.NT + g] = xn[d];
  a.logq[g] = lq;
  a.sel[g] = comp;
}

// Network on the current state of every stepping filter: one 16-row tile of
// outer particles per workgroup; rows of filters that sit the step out get
// zero features (their outputs are not used).  The epilogue draws each
// row's proposal from its mixture.
template <class Mdl>
__global__ __launch_bounds__(kBlock) void k_mlp_fwd_state(StepArgs a) {
  constexpr int NF = Mdl::DX + Mdl::DY + 2 * Mdl::DZ;
  static_assert(NF <= kMlpIn, "features do not fit the input layer");
  __shared__ MlpShared sh;
  MlpFrags fr;
  mlp_load_frags(a.mlp, fr);
  const int row0 = blockIdx.x * kMlpRows;
  const int nrows = min(kMlpRows, a.NT - row0);
  const float* fmean = reinterpret_cast<const float*>(a.mlp + MlpBlobLayout::fmean);
  const float* fstd = reinterpret_cast<const float*>(a.mlp + MlpBlobLayout::fstd);
  // The tile's features, two per thread: column c of row g is
  // [x_{t-1} (DX), y_t (DY), cloud mean (DZ), cloud variance (DZ)][c],
  // standardised.  Every load is issued at a clamped (in-range) index before
  // any value is used and the results are masked afterwards: a load guarded
  // by a branch would wait inside it, one memory round per guard.
  static_assert(kMlpRows * kMlpIn == 2 * kBlock, "two features per thread");
  constexpr int DX = Mdl::DX, DY = Mdl::DY, DZ = Mdl::DZ;
  float fv[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int e = threadIdx.x + q * kBlock;
    const int r = e / kMlpIn, c = e % kMlpIn;
    const int g = row0 + min(r, nrows - 1);
    const int f = filter_of_outer(a.ooff, a.n_filters, g);
    const int cc = min(c, NF - 1);
    const int am = a.active != nullptr ? a.active[f] : 1;
    const int tf = a.run_Tf != nullptr ? a.run_Tf[f] : 0x7fffffff;
    const int tc = a.tcur[f];
    const unsigned char cu = a.cur[f];
    const float mu = fmean[cc], sd = fstd[cc];
    const float* px = a.x[copy_of(cu)] + (long long)min(cc, DX - 1) * a.NT + g;
    // (a run's observation row, clamped: a filter past its horizon reads row
    // run_T - 1 and masks it)
    const int ty = a.y_tstride != 0 ? min(tc, a.run_T - 1) : 0;
    const float* py = a.Y + (long long)ty * a.y_tstride + (long long)f * DY + min(max(cc - DX, 0), DY - 1);
    const float* pm = a.mom + (long long)g * 2 * DZ + min(max(cc - DX - DY, 0), 2 * DZ - 1);
    const float raw = *(cc < DX ? px : (cc < DX + DY ? py : pm));
    const bool act = am != 0 && tc < min(tf, a.run_T);
    fv[q] = (r < nrows && c < NF && act) ? (raw - mu) / sd : 0.f;
  }
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int e = threadIdx.x + q * kBlock;
    sh.x0[e / kMlpIn][e % kMlpIn] = f2bf(fv[q]);
  }
  __syncthreads();
  mlp_rows<false>(fr, sh, row0, nrows, a.mdn, MlpTrainOut{});
  __syncthreads();
  if (threadIdx.x < nrows) {
    const int g = row0 + threadIdx.x;
    const int f = filter_of_outer(a.ooff, a.n_filters, g);
    if (step_active(a, f)) {
      float o[Mdn<Mdl::DX>::kUsed];
#pragma unroll
      for (int c = 0; c < Mdn<Mdl::DX>::kUsed; ++c) o[c] = sh.o[threadIdx.x][c];
      mdn_propose<Mdl::DX>(a, f, g, o);
    }
  }
}

// Proposals from caller-supplied mixture outputs (a.mdn), one thread per
// outer particle.
template <class Mdl>
__global__ __launch_bounds__(kBlock) void k_mdn_draw(StepArgs a) {
  const int g = blockIdx.x * kBlock + threadIdx.x;
  if (g >= a.NT) return;
  const int f = filter_of_outer(a.ooff, a.n_filters, g);
  if (!step_active(a, f)) return;
  float o[Mdn<Mdl::DX>::kUsed];
#pragma unroll
  for (int c = 0; c < Mdn<Mdl::DX>::kUsed; ++c) o[c] = a.mdn[(long long)g * kMlpOut + c];
  mdn_propose<Mdl::DX>(a, f, g, o);
}

// Proposal draw and inner pass of the learned step for one tile of outer
// particles (pre-resampling index i; results go to slot i of the next copy).
template <class Mdl, int SEG, int JPT>
__global__ __launch_bounds__(kBlock) void k_learned_inner(StepArgs a) {
  constexpr int DX = Mdl::DX, DZ = Mdl::DZ, DY = Mdl::DY;
  constexpr int NSEG = kBlock / SEG;
  constexpr bool kKeepZ = JPT * DZ <= 64;
  __shared__ SegScratch sh;
  __shared__ double cdf[NSEG][SEG * JPT];
  __shared__ float vred[kBlock / kWave][2 * DZ];

  const int4 tile = a.tiles[blockIdx.x];
  const int f = tile.x;
  const bool act = step_active(a, f);
  if (tile.z == 0 && threadIdx.x == 0) a.act[f] = act ? 1 : 0;
  if (!act) return;
  const int N = a.fN[f], M = a.fM[f];
  const int s = threadIdx.x / SEG;
  const int ls = threadIdx.x % SEG;
  const int i = tile.y + s;
  const bool vi = i < N;
  const int oo = a.ooff[f];
  const long long io = a.ioff[f];
  const int t = a.tcur[f] + 1;
  const unsigned char cb = a.cur[f];
  const int src = copy_of(cb), dst = src ^ 1;
  const Key key = make_key(a.seed, (uint32_t)f);
  const int ci = vi ? (ident_slots(cb, src) ? i : a.ind[src][oo + i]) : 0;

  float xp[DX];
#pragma unroll
  for (int d = 0; d < DX; ++d) xp[d] = vi ? a.x[src][(long long)d * a.NT + oo + i] : 0.f;
  const float* zp = a.z[src] + (io + (long long)ci * M) * DZ;
  const float* lp = a.lam[src] + io + (long long)ci * M;

  // ---- 1. x_t ~ q(. | features of particle i), drawn by the network's
  //         epilogue (or k_mdn_draw) -------------------------------------
  float xn[DX];
  const long long gi = oo + (vi ? i : 0);
#pragma unroll
  for (int d = 0; d < DX; ++d) xn[d] = a.xtmp[(long long)d * a.NT + gi];
  const float lq = a.logq[gi];

  // ---- 2. kappa = lam + log p(x_t | x_{t-1}, z) and its log-sum-exp ------
  float zd[DZ];
#pragma unroll
  for (int d = 0; d < DZ; ++d) zd[d] = 0.f;
  const float lpx0 = Mdl::kXdepZ ? 0.f : Mdl::logpx(as_prm(a.prm), xn, xp, zd, t - 1);
  float cpx[npx<Mdl>()];
  if constexpr (Mdl::kXdepZ) Mdl::px_pre(as_prm(a.prm), xn, xp, t - 1, cpx);
  float ev[JPT];
  float mk = -INFINITY;
#pragma unroll
  for (int r = 0; r < JPT; ++r) {
    const int j = ls + r * SEG;
    ev[r] = -INFINITY;
    if (vi && j < M) {
      float kap = lp[j];
      if constexpr (Mdl::kXdepZ) {
        float zj[DZ];
#pragma unroll
        for (int d = 0; d < DZ; ++d) zj[d] = zp[d * M + j];
        kap += Mdl::logpx_post(as_prm(a.prm), cpx, zj);
      } else {
        kap += lpx0;
      }
      ev[r] = kap;
      if (finitef(kap)) mk = fmaxf(mk, kap);
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
  __syncthreads();
  const double tot2 = cdf[s][M - 1];
  const float log_px = deg2 ? -INFINITY : m2 + fast_log((float)tot2);  // eq:approx1 at x_t
  const double u_in = uniform53(key, (uint32_t)t, (uint32_t)i, P_INNER_U);

  // ---- 3. local resampling, propagation, measurement update --------------
  float pre[Mdl::NPRE];
  fz_pre_seg<Mdl, SEG>(as_prm(a.prm), xp, xn, t - 1, pre);
  float y[DY], r0[DY];
  load_y<Mdl>(a, f, t, y);
  Mdl::obs_pre(as_prm(a.prm), y, xn, r0);
  float* zdst = a.z[dst] + (io + (long long)i * M) * DZ;
  float llv[JPT];
  float zkeep[kKeepZ ? JPT : 1][DZ];
  Lse acc;
#pragma unroll
  for (int r = 0; r < JPT; ++r) {
    const int jj = ls + r * SEG;
    llv[r] = -INFINITY;
    if (vi && jj < M) {
      const int b = cdf_search(cdf[s], M, sys_point(jj, u_in, tot2, M));
      float zg[DZ], nu[DZ], zn[DZ];
#pragma unroll
      for (int d = 0; d < DZ; ++d) zg[d] = zp[d * M + b];
      normals<DZ>(key, (uint32_t)t, (uint32_t)i, (uint32_t)jj, P_NEW_Z, nu);
      Mdl::fz_post(as_prm(a.prm), pre, zg, nu, zn);
#pragma unroll
      for (int d = 0; d < DZ; ++d) zdst[d * M + jj] = zn[d];
      if constexpr (kKeepZ) {
#pragma unroll
        for (int d = 0; d < DZ; ++d) zkeep[kKeepZ ? r : 0][d] = zn[d];
      }
      llv[r] = Mdl::logpy_post(as_prm(a.prm), r0, zn);
      acc.add(llv[r]);
    }
  }
  const float lse = seg_lse<SEG>(acc, sh);
  const bool deg3 = !(lse > -INFINITY);
  float* ldst = a.lam[dst] + io + (long long)i * M;
  float part[2 * DZ];
#pragma unroll
  for (int d = 0; d < 2 * DZ; ++d) part[d] = 0.f;
#pragma unroll
  for (int r = 0; r < JPT; ++r) {
    const int jj = ls + r * SEG;
    if (vi && jj < M) {
      const float lam = deg3 ? -fast_log((float)M) : (finitef(llv[r]) ? llv[r] - lse : -INFINITY);
      ldst[jj] = lam;
      const float q = deg3 ? 1.0f / (float)M : (finitef(llv[r]) ? fast_exp(lam) : 0.f);
#pragma unroll
      for (int d = 0; d < DZ; ++d) {
        const float zv = kKeepZ ? zkeep[kKeepZ ? r : 0][d] : zdst[d * M + jj];
        part[d] += q * zv;
        part[DZ + d] += q * zv * zv;
      }
    }
  }
  static_assert(2 * DZ <= 16, "moment vector too long for the transpose reduction");
  int slot;
  const float tot = seg_sum_vec_t<SEG, 2 * DZ>(part, vred, slot);
  const float mean = seg_vec_fetch<SEG, 2 * DZ>(tot, slot >= DZ ? slot - DZ : -1);
  if (vi && slot >= 0) {
    float* mp = a.mom_tmp + (long long)(oo + i) * 2 * DZ;
    if (slot < DZ) {
      a.kpart_tmp[(long long)(oo + i) * DZ + slot] = tot;
      mp[slot] = tot;
    } else {
      mp[slot] = fmaxf(tot - mean * mean, 0.f);
    }
  }
  if (vi && ls == 0) {
    // Fig. 2 step 1 weight: eq:approx2 (unit inner weights) x eq:approx1 / q
    const float log_py = deg3 ? -INFINITY : lse - fast_log((float)M);
    a.logw[oo + i] = (log_py + log_px) - lq;
    if (deg2 || deg3) atomicOr(&a.lflags[f], (uint32_t)F_DEGENERATE_INNER);
  }
}

// Exact (two-pass) qbar-weighted mean and variance of every particle's inner
// cloud in the current state copy -> mom [NT][2 DZ]; with feat != null also
// the raw feature rows [NT][32] for y = y_f (zero padded).
template <class Mdl, int SEG, int JPT>
__global__ __launch_bounds__(kBlock) void k_moments(StepArgs a, const float* y, float* feat) {
  constexpr int DX = Mdl::DX, DZ = Mdl::DZ, DY = Mdl::DY;
  constexpr int NSEG = kBlock / SEG;
  __shared__ float vred[kBlock / kWave][DZ];
  __shared__ float mean_sh[NSEG][DZ];
  const int4 tile = a.tiles[blockIdx.x];
  const int f = tile.x;
  const int N = a.fN[f], M = a.fM[f];
  const int s = threadIdx.x / SEG;
  const int ls = threadIdx.x % SEG;
  const int i = tile.y + s;
  const bool vi = i < N;
  const int oo = a.ooff[f];
  const long long io = a.ioff[f];
  const unsigned char cb = a.cur[f];
  const int c = copy_of(cb);
  const int ci = vi ? (ident_slots(cb, c) ? i : a.ind[c][oo + i]) : 0;
  const float* zp = a.z[c] + (io + (long long)ci * M) * DZ;
  const float* lp = a.lam[c] + io + (long long)ci * M;
  float part[DZ];
#pragma unroll
  for (int d = 0; d < DZ; ++d) part[d] = 0.f;
  for (int r = 0; r < JPT; ++r) {
    const int j = ls + r * SEG;
    if (vi && j < M) {
      const float q = fast_exp(lp[j]);
#pragma unroll
      for (int d = 0; d < DZ; ++d) part[d] += q * zp[d * M + j];
    }
  }
  seg_sum_vec<SEG, DZ>(part, vred);
  if (ls == 0) {
#pragma unroll
    for (int d = 0; d < DZ; ++d) mean_sh[s][d] = part[d];
  }
  __syncthreads();
  float mean[DZ];
#pragma unroll
  for (int d = 0; d < DZ; ++d) {
    mean[d] = mean_sh[s][d];
    part[d] = 0.f;
  }
  for (int r = 0; r < JPT; ++r) {
    const int j = ls + r * SEG;
    if (vi && j < M) {
      const float q = fast_exp(lp[j]);
#pragma unroll
      for (int d = 0; d < DZ; ++d) {
        const float e = zp[d * M + j] - mean[d];
        part[d] += q * e * e;
      }
    }
  }
  seg_sum_vec<SEG, DZ>(part, vred);
  if (vi && ls == 0) {
    const long long g = oo + i;
#pragma unroll
    for (int d = 0; d < DZ; ++d) {
      a.mom[g * 2 * DZ + d] = mean[d];
      a.mom[g * 2 * DZ + DZ + d] = part[d];
    }
    if constexpr (DX + DY + 2 * DZ <= kMlpIn) {
      if (feat) {
        float* fr = feat + g * kMlpIn;
      int q = 0;
#pragma unroll
      for (int d = 0; d < DX; ++d) fr[q++] = a.x[c][(long long)d * a.NT + g];
#pragma unroll
      for (int d = 0; d < DY; ++d) fr[q++] = y[(long long)f * DY + d];
#pragma unroll
      for (int d = 0; d < DZ; ++d) fr[q++] = mean[d];
#pragma unroll
      for (int d = 0; d < DZ; ++d) fr[q++] = part[d];
        for (; q < kMlpIn; ++q) fr[q] = 0.f;
      }
    }
  }
}

}  // namespace dpf
