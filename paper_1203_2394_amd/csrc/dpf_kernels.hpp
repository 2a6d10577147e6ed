// Step kernels of the look-ahead DPF (Section 2.2, Fig. 4) and of the plain
// DPF (Section 2, Fig. 2) for many independent filters of uneven sizes.
//
// Data layout in HBM (filter f, outer offset oo = ooff[f], inner offset
// io = ioff[f], sizes N = fN[f], M = fM[f]):
//   x    [DX][NT]            x[d * NT + oo + i]          (SoA, coalesced over i)
//   z    [sum N*DZ*M]         z[(io + i*M) * DZ + d*M + j] ([N][DZ][M] per filter)
//   lam  [sum N*M]            lam[io + i*M + j]           (log qbar, eq:qbar)
//   ell  [sum N*M]            look-ahead / measurement log-weights
//   logw [NT], anc [NT], kpart [NT][DZ], cdf [NT] (FP64)
// x, z and lam are double-buffered; cur[f] says which copy holds the state of
// filter f, so filters that sit a step out keep their state without a copy.
//
// Per-particle kernels run one 256-thread workgroup per tile of 256/SEG
// consecutive outer particles of one filter (a "segment" of SEG lanes per
// particle, lane l handling inner indices l, l+SEG, ..., up to SEG*JPT).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "dpf_models.hpp"
#include "dpf_rng.hpp"
#include "dpf_seg.hpp"

namespace dpf {

enum FlagBits : uint32_t {
  F_DEGENERATE_OUTER = 1u,
  F_DEGENERATE_INNER = 2u,
  F_NONFINITE = 4u,
  F_FALLBACK = 8u
};

struct StepArgs {
  const float* prm;
  const int2* tiles;  // (filter, first outer index)
  const int* fN;
  const int* fM;
  const int* ooff;
  const long long* ioff;
  int NT;
  int t_offset;  // counter time = tcur[f] + t_offset
  uint64_t seed;
  int* tcur;
  unsigned char* cur;
  const unsigned char* active;
  const float* Y;
  long long y_tstride;  // y of filter f at time t: Y + (t-1) * y_tstride + f * DY
  float* x[2];
  float* z[2];
  float* lam[2];
  float* ell;
  float* logw;
  int* anc;
  int* sel;      // [NT] selected candidate (look-ahead) / inner ancestor (plain)
  float* kpart;  // [NT][DZ]
  float* mom;    // [NT][2*DZ] or null: qbar-weighted moments of each new cloud
  double* cdf;   // [NT]
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
};

__device__ __forceinline__ bool filter_active(const StepArgs& a, int f) {
  return a.active == nullptr || a.active[f] != 0;
}

template <class Mdl>
__device__ __forceinline__ void load_y(const StepArgs& a, int f, int t, float* y) {
  const float* yp = a.Y + (long long)(t - 1) * a.y_tstride + (long long)f * Mdl::DY;
#pragma unroll
  for (int k = 0; k < Mdl::DY; ++k) y[k] = yp[k];
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

// ------------------------------------------------------------ initialisation
// Prior draws [x_0; z_0] ~ N(0, I) (INIT_X at (0, i, 0), INIT_Z at (0, i, j)).
// Look-ahead state: lam_0 = -log M, written to copy 0.  Plain DPF: the prior
// goes to copy 1 with ell = 0 and anc = identity, after which the proposal
// kernel runs with t = 0 (no y_0 is consumed).
template <class Mdl, int SEG, int JPT, bool PLAIN>
__global__ __launch_bounds__(kBlock) void k_init(StepArgs a) {
  const int2 tile = a.tiles[blockIdx.x];
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
template <class Mdl, int SEG, int JPT>
__global__ __launch_bounds__(kBlock) void k_la_weights(StepArgs a) {
  __shared__ SegScratch sh;
  const int2 tile = a.tiles[blockIdx.x];
  const int f = tile.x;
  if (!filter_active(a, f)) return;
  const int N = a.fN[f], M = a.fM[f];
  const int i = tile.y + threadIdx.x / SEG;
  const int ls = threadIdx.x % SEG;
  const bool vi = i < N;
  const int oo = a.ooff[f];
  const long long io = a.ioff[f];
  const int t = a.tcur[f] + a.t_offset;
  const int src = a.cur[f];
  const Key key = make_key(a.seed, (uint32_t)f);

  float y[Mdl::DY], x[Mdl::DX];
  load_y<Mdl>(a, f, t, y);
#pragma unroll
  for (int d = 0; d < Mdl::DX; ++d) x[d] = vi ? a.x[src][(long long)d * a.NT + oo + i] : 0.f;

  const float* zrow = a.z[src] + (io + (long long)(vi ? i : 0) * M) * Mdl::DZ;
  const float* lrow = a.lam[src] + io + (long long)(vi ? i : 0) * M;
  float* erow = a.ell + io + (long long)(vi ? i : 0) * M;
  Lse acc;
#pragma unroll
  for (int r = 0; r < JPT; ++r) {
    const int j = ls + r * SEG;
    if (vi && j < M) {
      float z[Mdl::DZ], nu_x[Mdl::DX], nu_z[Mdl::DZ], xl[Mdl::DX], pre[Mdl::DZ], zl[Mdl::DZ],
          r0[Mdl::DY];
#pragma unroll
      for (int d = 0; d < Mdl::DZ; ++d) z[d] = zrow[d * M + j];
      const float lam = lrow[j];
      normals<Mdl::DX>(key, (uint32_t)t, (uint32_t)i, (uint32_t)j, P_LA_X, nu_x);
      normals<Mdl::DZ>(key, (uint32_t)t, (uint32_t)i, (uint32_t)j, P_LA_Z, nu_z);
      Mdl::fx(a.prm, x, z, nu_x, xl);
      Mdl::fz_pre(a.prm, x, xl, pre);
      Mdl::fz_post(a.prm, pre, z, nu_z, zl);
      Mdl::obs_pre(a.prm, y, xl, r0);
      const float e = lam + Mdl::logpy_post(a.prm, r0, zl);
      erow[j] = e;
      acc.add(e);
    }
  }
  const float lw = seg_lse<SEG>(acc, sh);
  if (vi && ls == 0) a.logw[oo + i] = lw;
}

// --------------------------------------------------------- plain weights
// Fig. 2 step 1 (eq:approx2 with unit inner weights): ell = log p(y_t | xt, zt),
// log w_i = logsumexp_j ell - log M, and the per-particle partial
// sum_j qbar_ij zt_ij (qbar = softmax_j ell, step 3) for the estimate.
template <class Mdl, int SEG, int JPT>
__global__ __launch_bounds__(kBlock) void k_dpf_weights(StepArgs a) {
  __shared__ SegScratch sh;
  const int2 tile = a.tiles[blockIdx.x];
  const int f = tile.x;
  if (!filter_active(a, f)) return;
  const int N = a.fN[f], M = a.fM[f];
  const int i = tile.y + threadIdx.x / SEG;
  const int ls = threadIdx.x % SEG;
  const bool vi = i < N;
  const int oo = a.ooff[f];
  const long long io = a.ioff[f];
  const int t = a.tcur[f] + a.t_offset;
  const int src = a.cur[f];

  float y[Mdl::DY], x[Mdl::DX], r0[Mdl::DY];
  load_y<Mdl>(a, f, t, y);
#pragma unroll
  for (int d = 0; d < Mdl::DX; ++d) x[d] = vi ? a.x[src][(long long)d * a.NT + oo + i] : 0.f;
  Mdl::obs_pre(a.prm, y, x, r0);
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
      ev[r] = Mdl::logpy_post(a.prm, r0, z);
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
#pragma unroll
  for (int d = 0; d < Mdl::DZ; ++d) part[d] = seg_sum<SEG>(part[d], sh);
  if (vi && ls == 0) {
    a.logw[oo + i] = deg ? -INFINITY : lse - fast_log((float)M);
#pragma unroll
    for (int d = 0; d < Mdl::DZ; ++d) a.kpart[(long long)(oo + i) * Mdl::DZ + d] = part[d];
    if (deg) atomicOr(&a.flags[f], (uint32_t)F_DEGENERATE_INNER);
  }
}

// -------------------------------------------------------- outer resampling
// One 1024-thread workgroup per filter.  Weights w_i = exp(log w_i - max)
// (FP32 exponent, widened), FP64 inclusive scan (serial within a chunk of
// consecutive indices per thread, then across chunks), systematic points
// ((k + u) * C) / N with u = U53 at (t, 0, 0) of OUTER_U, first index with
// C_i > point.  Also ESS = C^2 / sum w^2 and dlogZ = max + log C - log N.
constexpr int kResBlock = 1024;

struct ResScratch {
  double part[kResBlock];
  float fred[kResBlock / kWave];
  double dred[kResBlock / kWave];
};

__device__ __forceinline__ float block_max_1024(float v, ResScratch& sh) {
  for (int off = kWave / 2; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, kWave));
  if ((threadIdx.x & (kWave - 1)) == 0) sh.fred[threadIdx.x / kWave] = v;
  __syncthreads();
  float r = sh.fred[0];
  for (int q = 1; q < kResBlock / kWave; ++q) r = fmaxf(r, sh.fred[q]);
  __syncthreads();
  return r;
}

__device__ __forceinline__ double block_sum_1024(double v, ResScratch& sh) {
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) sh.dred[threadIdx.x / kWave] = v;
  __syncthreads();
  double r = 0.0;
  for (int q = 0; q < kResBlock / kWave; ++q) r += sh.dred[q];
  __syncthreads();
  return r;
}

// In-place FP64 inclusive scan of C[0..n) by one 1024-thread block.
__device__ void block_scan_inplace(double* C, int n, ResScratch& sh) {
  const int ch = (n + kResBlock - 1) / kResBlock;
  const int lo = threadIdx.x * ch;
  const int hi = min(lo + ch, n);
  double s = 0.0;
  for (int q = lo; q < hi; ++q) s += C[q];
  sh.part[threadIdx.x] = s;
  __syncthreads();
  // exclusive scan of chunk sums (Hillis-Steele over the 1024 partials)
  for (int d = 1; d < kResBlock; d <<= 1) {
    const double o = (threadIdx.x >= d) ? sh.part[threadIdx.x - d] : 0.0;
    __syncthreads();
    sh.part[threadIdx.x] += o;
    __syncthreads();
  }
  double run = (threadIdx.x > 0) ? sh.part[threadIdx.x - 1] : 0.0;
  for (int q = lo; q < hi; ++q) {
    run += C[q];
    C[q] = run;
  }
  __syncthreads();
}

__device__ void block_systematic(const double* C, int n, int n_out, double u, int* out) {
  const double total = C[n - 1];
  for (int k = threadIdx.x; k < n_out; k += kResBlock) out[k] = cdf_search(C, n, sys_point(k, u, total, n_out));
}

__global__ __launch_bounds__(kResBlock) void k_outer_resample(StepArgs a) {
  __shared__ ResScratch sh;
  const int f = blockIdx.x;
  if (!filter_active(a, f)) return;
  const int N = a.fN[f];
  const int oo = a.ooff[f];
  const int t = a.tcur[f] + a.t_offset;
  const float* lw = a.logw + oo;
  double* C = a.cdf + oo;

  float m = -INFINITY;
  bool nonf = false;
  for (int i = threadIdx.x; i < N; i += kResBlock) {
    const float v = lw[i];
    if (finitef(v))
      m = fmaxf(m, v);
    else if (!(v == -INFINITY))
      nonf = true;
  }
  m = block_max_1024(m, sh);
  const bool deg = !(m > -INFINITY);
  double sq = 0.0;
  for (int i = threadIdx.x; i < N; i += kResBlock) {
    const float v = lw[i];
    const double w = deg ? 1.0 : (finitef(v) ? (double)fast_exp(v - m) : 0.0);
    C[i] = w;
    sq += w * w;
  }
  sq = block_sum_1024(sq, sh);
  const int any_nonf = __syncthreads_or(nonf ? 1 : 0);
  block_scan_inplace(C, N, sh);
  const double total = C[N - 1];
  const Key key = make_key(a.seed, (uint32_t)f);
  const double u = uniform53(key, (uint32_t)t, 0u, P_OUTER_U);
  block_systematic(C, N, N, u, a.anc + oo);
  if (threadIdx.x == 0) {
    a.fstat[4 * f + 0] = deg ? 0.0 : (double)m;
    a.fstat[4 * f + 1] = total;
    a.fstat[4 * f + 2] = sq;
    a.fstat[4 * f + 3] = deg ? 1.0 : 0.0;
    a.ess[f] = (float)(total * total / sq);
    const double dl = deg ? -INFINITY : (double)m + log(total) - log((double)N);
    a.dlogz[f] = dl;
    a.loglik[f] += dl;
    uint32_t fl = 0;
    if (deg) fl |= F_DEGENERATE_OUTER;
    if (any_nonf) fl |= F_NONFINITE;
    const float* yp = a.Y + (long long)(t - 1) * a.y_tstride + (long long)f * a.dy;
    for (int q = 0; q < a.dy; ++q)
      if (!finitef(yp[q])) fl |= F_NONFINITE;
    if (fl) atomicOr(&a.flags[f], fl);
  }
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
__global__ __launch_bounds__(kBlock) void k_newcloud(StepArgs a) {
  constexpr int DX = Mdl::DX, DZ = Mdl::DZ, DY = Mdl::DY;
  constexpr int NSEG = kBlock / SEG;
  __shared__ SegScratch sh;
  __shared__ double cdf[NSEG][SEG * JPT];
  __shared__ float xs_sh[NSEG][DX];
  __shared__ int csel[NSEG];

  const int2 tile = a.tiles[blockIdx.x];
  const int f = tile.x;
  if (!filter_active(a, f)) return;
  const int N = a.fN[f], M = a.fM[f];
  const int s = threadIdx.x / SEG;
  const int ls = threadIdx.x % SEG;
  const int k = tile.y + s;
  const bool vk = k < N;
  const int oo = a.ooff[f];
  const long long io = a.ioff[f];
  const int t = a.tcur[f] + a.t_offset;
  const int src = a.cur[f], dst = src ^ 1;
  const Key key = make_key(a.seed, (uint32_t)f);
  const int p = vk ? a.anc[oo + k] : 0;

  float xp[DX];
#pragma unroll
  for (int d = 0; d < DX; ++d) xp[d] = a.x[src][(long long)d * a.NT + oo + p];
  const float* zp = a.z[src] + (io + (long long)p * M) * DZ;
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
  const bool deg1 = !(m1 > -INFINITY);
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
  const int c = csel[s];

  // ---- 2. the new outer particle ----------------------------------------
  if (ls == 0) {
    float zc[DZ], nu[DX], xn[DX];
#pragma unroll
    for (int d = 0; d < DZ; ++d) zc[d] = zp[d * M + c];
    if (PLAIN)
      normals<DX>(key, (uint32_t)t, (uint32_t)k, 0u, P_DPF_X, nu);
    else
      normals<DX>(key, (uint32_t)t, (uint32_t)p, (uint32_t)c, P_LA_X, nu);
    Mdl::fx(a.prm, xp, zc, nu, xn);
#pragma unroll
    for (int d = 0; d < DX; ++d) xs_sh[s][d] = xn[d];
    if (vk) {
#pragma unroll
      for (int d = 0; d < DX; ++d) a.x[dst][(long long)d * a.NT + oo + k] = xn[d];
    }
  }
  __syncthreads();
  float xn[DX];
#pragma unroll
  for (int d = 0; d < DX; ++d) xn[d] = xs_sh[s][d];

  // ---- 3. x-conditioned inner weights and local systematic resampling ---
  const float* lp = a.lam[src] + io + (long long)p * M;
  float mk = -INFINITY;
#pragma unroll
  for (int r = 0; r < JPT; ++r) {
    const int j = ls + r * SEG;
    if (vk && j < M) {
      float kap = PLAIN ? ev[r] : lp[j];
      if (Mdl::kXdepZ) {
        float zj[DZ];
#pragma unroll
        for (int d = 0; d < DZ; ++d) zj[d] = zp[d * M + j];
        kap += Mdl::logpx(a.prm, xn, xp, zj);
      }
      ev[r] = kap;
      if (finitef(kap)) mk = fmaxf(mk, kap);
    } else {
      ev[r] = -INFINITY;
    }
  }
  const float m2 = seg_max<SEG>(mk, sh);
  const bool deg2 = !(m2 > -INFINITY);
  carry = 0.0;
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
  const double u_in = uniform53(key, (uint32_t)t, (uint32_t)k, P_INNER_U);
  const double tot2 = cdf[s][M - 1];

  // ---- 4. gather + propagate (+ measurement update in look-ahead mode) ---
  float pre[DZ];
  Mdl::fz_pre(a.prm, xp, xn, pre);
  float y[DY], r0[DY];
  if (!PLAIN) {
    load_y<Mdl>(a, f, t, y);
    Mdl::obs_pre(a.prm, y, xn, r0);
  }
  float* zdst = a.z[dst] + (io + (long long)k * M) * DZ;
  float llv[JPT];
  Lse acc;
#pragma unroll
  for (int r = 0; r < JPT; ++r) {
    const int jj = ls + r * SEG;
    llv[r] = -INFINITY;
    if (vk && jj < M) {
      const int b = cdf_search(cdf[s], M, sys_point(jj, u_in, tot2, M));
      float zg[DZ], nu[DZ], zn[DZ];
#pragma unroll
      for (int d = 0; d < DZ; ++d) zg[d] = zp[d * M + b];
      normals<DZ>(key, (uint32_t)t, (uint32_t)k, (uint32_t)jj, PLAIN ? P_DPF_Z : P_NEW_Z, nu);
      Mdl::fz_post(a.prm, pre, zg, nu, zn);
#pragma unroll
      for (int d = 0; d < DZ; ++d) zdst[d * M + jj] = zn[d];
      if (!PLAIN) {
        llv[r] = Mdl::logpy_post(a.prm, r0, zn);
        acc.add(llv[r]);
      }
    }
  }
  uint32_t fl = (deg1 || deg2) ? (uint32_t)F_DEGENERATE_INNER : 0u;
  if (!PLAIN) {
    const float lse = seg_lse<SEG>(acc, sh);
    const bool deg3 = !(lse > -INFINITY);
    if (deg3) fl |= F_DEGENERATE_INNER;
    float* ldst = a.lam[dst] + io + (long long)k * M;
    float part[DZ], part2[DZ];
#pragma unroll
    for (int d = 0; d < DZ; ++d) part[d] = part2[d] = 0.f;
#pragma unroll
    for (int r = 0; r < JPT; ++r) {
      const int jj = ls + r * SEG;
      if (vk && jj < M) {
        const float lam = deg3 ? -fast_log((float)M) : (finitef(llv[r]) ? llv[r] - lse : -INFINITY);
        ldst[jj] = lam;
        const float q = deg3 ? 1.0f / (float)M : (finitef(llv[r]) ? fast_exp(lam) : 0.f);
#pragma unroll
        for (int d = 0; d < DZ; ++d) {
          const float zv = zdst[d * M + jj];
          part[d] += q * zv;
          part2[d] += q * zv * zv;
        }
      }
    }
#pragma unroll
    for (int d = 0; d < DZ; ++d) part[d] = seg_sum<SEG>(part[d], sh);
    if (a.mom != nullptr) {
#pragma unroll
      for (int d = 0; d < DZ; ++d) part2[d] = seg_sum<SEG>(part2[d], sh);
    }
    if (vk && ls == 0) {
#pragma unroll
      for (int d = 0; d < DZ; ++d) a.kpart[(long long)(oo + k) * DZ + d] = part[d];
      if (a.mom != nullptr) {
#pragma unroll
        for (int d = 0; d < DZ; ++d) {
          a.mom[(long long)(oo + k) * 2 * DZ + d] = part[d];
          a.mom[(long long)(oo + k) * 2 * DZ + DZ + d] = fmaxf(part2[d] - part[d] * part[d], 0.f);
        }
      }
    }
  }
  if (vk && ls == 0 && fl) atomicOr(&a.flags[f], fl);
}

// ---------------------------------------------------------------- estimates
// One workgroup per filter; FP64 sums in a fixed order (strided per thread,
// then a fixed tree), so results are reproducible run to run.
//   look-ahead: xhat = mean_k x_t^(k), zhat = mean_k sum_j qbar z
//   plain:      xhat = sum_i Wbar_i xt_i, zhat = sum_i Wbar_i sum_j qbar z
// Then the state copy flips and the filter's time advances.
template <int DX, int DZ, bool PLAIN>
__global__ __launch_bounds__(kBlock) void k_finalize(StepArgs a, int advance) {
  __shared__ double red[DX + DZ][kBlock / kWave];
  const int f = blockIdx.x;
  if (!filter_active(a, f)) return;
  const int N = a.fN[f];
  const int oo = a.ooff[f];
  const int src = a.cur[f];
  const int t = a.tcur[f] + a.t_offset;
  if (advance) {
    const float* xs = PLAIN ? a.x[src] : a.x[src ^ 1];
    double mx = 0.0, tot = 1.0;
    if (PLAIN) {
      mx = a.fstat[4 * f + 0];
      tot = a.fstat[4 * f + 1];
    }
    const bool deg = PLAIN && a.fstat[4 * f + 3] != 0.0;
    double acc[DX + DZ];
#pragma unroll
    for (int q = 0; q < DX + DZ; ++q) acc[q] = 0.0;
    for (int i = threadIdx.x; i < N; i += kBlock) {
      double w;
      if (PLAIN) {
        const float lw = a.logw[oo + i];
        w = finitef(lw) ? (double)fast_exp((float)((double)lw - mx)) / tot : 0.0;
        if (deg) w = 1.0 / N;
      } else {
        w = 1.0 / N;
      }
#pragma unroll
      for (int d = 0; d < DX; ++d) acc[d] += w * (double)xs[(long long)d * a.NT + oo + i];
#pragma unroll
      for (int d = 0; d < DZ; ++d) acc[DX + d] += w * (double)a.kpart[(long long)(oo + i) * DZ + d];
    }
#pragma unroll
    for (int q = 0; q < DX + DZ; ++q) {
      double v = acc[q];
      for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
      if ((threadIdx.x & (kWave - 1)) == 0) red[q][threadIdx.x / kWave] = v;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < DX + DZ; q += kBlock) {
      double v = 0.0;
      for (int w = 0; w < kBlock / kWave; ++w) v += red[q][w];
      if (q < DX) {
        a.est_x[f * DX + q] = (float)v;
        if (a.trace_x) a.trace_x[((long long)(t - 1) * a.n_filters + f) * DX + q] = (float)v;
      } else {
        a.est_z[f * DZ + q - DX] = (float)v;
        if (a.trace_z) a.trace_z[((long long)(t - 1) * a.n_filters + f) * DZ + q - DX] = (float)v;
      }
    }
  }
  if (threadIdx.x == 0) {
    a.cur[f] = (unsigned char)(src ^ 1);
    if (advance) a.tcur[f] = a.tcur[f] + 1;
  }
}

}  // namespace dpf
