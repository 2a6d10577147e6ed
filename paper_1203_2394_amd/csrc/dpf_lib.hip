// Host side of libdpf.so: the C interface of include/dpf.h.
//
// A handle owns host state only.  dpf_create validates the config, carves
// the caller's device workspace into the buffers of the step kernels,
// uploads the parameters (converted to FP32 plus derived constants computed
// in FP64), builds the tile lists and queues the initialisation.  Each step
// call queues a fixed sequence of launches on the handle's stream; nothing
// synchronises with the host.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/dpf.h"
#include "dpf_aux.hpp"
#include "dpf_engine.hpp"
#include "dpf_kernels.hpp"
#include "dpf_learned.hpp"
#include "dpf_mlp.hpp"

using namespace dpf;

static thread_local std::string g_err;
thread_local MomArgs dpf::g_mom_args = {nullptr, nullptr};

dpf_status dpf::fail(dpf_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

extern "C" const char* dpf_last_error(void) { return g_err.c_str(); }

static int class_of(int M) {
  for (int c = 0; c < kNumDefaultClasses; ++c)
    if (M <= kClasses[c].seg * kClasses[c].jpt) return c;
  return -1;
}

static const Engine* find_engine(int model, int dx, int dz, int dy) {
  const Engine* e = nullptr;
  if (model == DPF_MODEL_LINGAUSS) e = &kEngLinGauss;
  if (model == DPF_MODEL_NONLIN) e = &kEngNonLin;
  if (model == DPF_MODEL_HIGHDIM) e = &kEngHighDim;
  if (model == DPF_MODEL_TWODIM) e = &kEngTwoDim;
  if (model == DPF_MODEL_FOURDIM) e = &kEngFourDim;
  if (model == DPF_MODEL_TWODIM_ZFIRST) e = &kEngTwoDimZ;
  if (!e || e->dx != dx || e->dz != dz || e->dy != dy) return nullptr;
  return e;
}

// ---------------------------------------------------------------- layout
struct Layout {
  size_t total = 0;
  size_t prm, fN, fM, ooff, ooff64, ioff, finfo, tcur, cur, act, tiles, rgroups, ginfo, x0, x1, z0, z1, l0, l1, ell,
      logw, anc, sel, kpart, gstat, fstat, ess, dlogz, loglik, flags, est_x, est_z;
  // slot indirection and learned-proposal buffers
  size_t ind0, ind1, mom, mlp, mdn, xtmp, logq, kpart_tmp, mom_tmp, fb, lflags;
  // second weight buffers: a look-ahead run alternates between the two
  size_t ell1, logw1;
  // step-end kernel: per-group partial estimates, per-filter counters
  size_t gpart, fcount;
  // Rao-Blackwellised estimate: per-outer partial sums
  size_t xrb;
  // predicted observation: per-outer partial sums (two, like ell) and [F]
  size_t yp0, yp1, est_y;
  int NT = 0;
  long long NMT = 0;
  int n_tiles = 0, n_rgroups = 0;
};

static size_t carve(size_t& cursor, size_t bytes) {
  const size_t off = cursor;
  cursor += (bytes + 255) & ~(size_t)255;
  return off;
}

static dpf_status plan(const dpf_config* c, const Engine*& eng, Layout& L) {
  if (!c) return fail(DPF_EINVAL, "config is NULL");
  if (c->abi_version != DPF_ABI_VERSION)
    return fail(DPF_EINVAL, "abi_version %u, library is %u", c->abi_version, DPF_ABI_VERSION);
  if (c->reserved != 0) return fail(DPF_EINVAL, "reserved field must be 0");
  if (c->algo != DPF_ALGO_LOOKAHEAD && c->algo != DPF_ALGO_PLAIN)
    return fail(DPF_EINVAL, "unknown algo %d", c->algo);
  eng = find_engine(c->model, c->dx, c->dz, c->dy);
  if (!eng)
    return fail(DPF_EUNSUPPORTED, "model %d with dims (%d,%d,%d) is not built", c->model, c->dx, c->dz,
                c->dy);
  if (!c->params || c->n_params != eng->n_raw)
    return fail(DPF_EINVAL, "model %d needs %zu parameters, got %zu", c->model, eng->n_raw, c->n_params);
  if (c->model == DPF_MODEL_TWODIM || c->model == DPF_MODEL_TWODIM_ZFIRST) {
    const double qx = c->params[0], qz = c->params[1], cxz = c->params[2], r = c->params[7];
    if (!(qx > 0.0 && qz > 0.0 && r > 0.0 && qz * qx > cxz * cxz))
      return fail(DPF_EINVAL, "TWODIM needs qx, qz, r > 0 and a positive definite noise covariance");
  }
  if (c->model == DPF_MODEL_FOURDIM) {
    const double* q = c->params;
    if (!(q[4] > 0.0 && q[5] > 0.0 && q[6] > 0.0 && q[13] > 0.0 && q[6] * q[7] > q[8] * q[8]))
      return fail(DPF_EINVAL, "FOURDIM needs positive variances and a positive definite inner noise covariance");
  }
  if (c->n_filters < 1 || !c->N || !c->M) return fail(DPF_EINVAL, "need n_filters >= 1 and N, M arrays");
  const int F = c->n_filters;
  L.NT = 0;
  L.NMT = 0;
  L.n_rgroups = 0;
  L.n_tiles = 0;  // room for any class: at most one tile per outer particle
  for (int f = 0; f < F; ++f) {
    if (c->N[f] < 1 || c->N[f] > 65536) return fail(DPF_EUNSUPPORTED, "N[%d] = %d outside 1..65536", f, c->N[f]);
    const int cls = class_of(c->M[f]);
    if (c->M[f] < 1 || cls < 0) return fail(DPF_EUNSUPPORTED, "M[%d] = %d outside 1..4096", f, c->M[f]);
    if ((long long)L.NT + c->N[f] > 0x7fffffffLL) return fail(DPF_EUNSUPPORTED, "total N too large");
    L.NT += c->N[f];
    L.NMT += (long long)c->N[f] * c->M[f];
    L.n_tiles += c->N[f];  // at most one tile per outer particle (SEG = 256)
    const int G = (c->N[f] + kResGroup - 1) / kResGroup;
    L.n_rgroups += G;
  }
  const int dx = c->dx, dz = c->dz;
  const size_t NT = L.NT, NMT = (size_t)L.NMT;
  size_t cur = 0;
  L.prm = carve(cur, eng->n_total * 4);
  L.fN = carve(cur, F * 4);
  L.fM = carve(cur, F * 4);
  L.ooff = carve(cur, (F + 1) * 4);
  L.ooff64 = carve(cur, (F + 1) * 8);
  L.ioff = carve(cur, (F + 1) * 8);
  L.finfo = carve(cur, F * sizeof(FilterInfo));
  L.tcur = carve(cur, F * 4);
  L.cur = carve(cur, F);
  L.act = carve(cur, F);
  L.tiles = carve(cur, (size_t)L.n_tiles * sizeof(int4));
  L.rgroups = carve(cur, (size_t)L.n_rgroups * sizeof(int2));
  L.ginfo = carve(cur, (size_t)L.n_rgroups * sizeof(int4));
  L.x0 = carve(cur, NT * dx * 4);
  L.x1 = carve(cur, NT * dx * 4);
  L.z0 = carve(cur, NMT * dz * 4);
  L.z1 = carve(cur, NMT * dz * 4);
  L.l0 = carve(cur, NMT * 4);
  L.l1 = carve(cur, NMT * 4);
  L.ell = carve(cur, NMT * 4);
  L.logw = carve(cur, NT * 4);
  L.ell1 = carve(cur, NMT * 4);
  L.logw1 = carve(cur, NT * 4);
  L.anc = carve(cur, NT * 4);
  L.sel = carve(cur, NT * 4);
  L.kpart = carve(cur, NT * dz * 4);
  // (a wave reads the statistics of 64 groups from the filter's first on,
  // whatever the filter's count: padded so those reads stay inside)
  L.gstat = carve(cur, ((size_t)L.n_rgroups + kWave) * 4 * 8);
  L.fstat = carve(cur, F * 4 * 8);
  L.ess = carve(cur, F * 4);
  L.dlogz = carve(cur, F * 8);
  L.loglik = carve(cur, F * 8);
  L.flags = carve(cur, F * 4);
  L.est_x = carve(cur, F * dx * 4);
  L.est_z = carve(cur, F * dz * 4);
  L.ind0 = carve(cur, NT * 4);
  L.ind1 = carve(cur, NT * 4);
  L.mom = carve(cur, NT * 2 * dz * 4);
  L.mlp = carve(cur, MlpBlobLayout::bytes);
  L.mdn = carve(cur, NT * kMlpOut * 4);
  L.xtmp = carve(cur, NT * dx * 4);
  L.logq = carve(cur, NT * 4);
  L.kpart_tmp = carve(cur, NT * dz * 4);
  L.mom_tmp = carve(cur, NT * 2 * dz * 4);
  L.fb = carve(cur, F);
  L.lflags = carve(cur, F * 4);
  L.gpart = carve(cur, (size_t)L.n_rgroups * (dx + dz + 1) * 8);
  L.fcount = carve(cur, F * 4);
  L.xrb = carve(cur, (size_t)L.NT * dx * 8);
  L.yp0 = carve(cur, NT * 4);
  L.yp1 = carve(cur, NT * 4);
  L.est_y = carve(cur, F * 4);
  L.total = cur;
  return DPF_OK;
}

// ---------------------------------------------------------------- tiling
struct dpf_handle;
static dpf_status build_tiles(dpf_handle* h);
// ---------------------------------------------------------------- handle
struct dpf_handle {
  const Engine* eng;
  int model, algo, dx, dz, dy, F;
  uint64_t seed;
  hipStream_t stream;
  Layout L;
  char* ws;
  std::vector<int> N, M, ooff;
  std::vector<long long> ioff, ooff64;
  std::vector<int4> tiles_h;
  std::vector<int2> rgroups_h;
  std::vector<int4> ginfo_h;  // per group: the filter's (first outer index, N, first group, groups)
  std::vector<FilterInfo> finfo_h;
  std::vector<float> prm_h;
  std::vector<TileClass> classes;
  std::vector<int> fcls;  // tile class of each filter
  // multi-step graph cache
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipGraphExec_t gexec_tail = nullptr;  // the run's last (T - 1) mod S steps
  const void* g_key[11] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                           nullptr, nullptr, nullptr, nullptr, nullptr};
  int g_T = -1;
  // phase timing: caller-owned events consumed kPhaseEvents per step
  std::vector<hipEvent_t> prof_events;
  size_t prof_next = 0;
  // learned proposal
  bool has_proposal = false;  // a network blob was set
  bool mom_valid = false;     // mom holds the moments of the current state
  double ess_frac = 0.1;
  // which weight buffers (0: ell/logw, 1: ell1/logw1) hold the weights of
  // the last step taken
  int ell_sel = 0;
  // the last call that changed the state was dpf_lookahead_step (what
  // dpf_estimate_rb needs)
  bool rb_ready = false;
  // companions per look-ahead candidate (nested estimator); 0: paired
  int n_comp = 0;
  // look-ahead steps form the predicted observation (and record it in ytrace)
  bool predict = false;
  float* ytrace = nullptr;
};

constexpr int kPhaseEvents = 5;
constexpr int kMaxCompanions = 1024;

// Drop the cached run graphs (their captured arguments are out of date).
static void drop_graphs(dpf_handle* h) {
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  if (h->gexec_tail) (void)hipGraphExecDestroy(h->gexec_tail);
  h->gexec = nullptr;
  h->gexec_tail = nullptr;
}

static dpf_status phase_mark(dpf_handle* h, int phase) {
  if (h->prof_next + (size_t)(kPhaseEvents - phase) > h->prof_events.size()) return DPF_OK;
  const hipError_t e = hipEventRecord(h->prof_events[h->prof_next], h->stream);
  h->prof_next++;
  if (e != hipSuccess) return fail(DPF_EDEVICE, "hipEventRecord of phase event: %s", hipGetErrorString(e));
  return DPF_OK;
}

template <class T>
static T* at(dpf_handle* h, size_t off) {
  return reinterpret_cast<T*>(h->ws + off);
}

static StepArgs make_args(dpf_handle* h) {
  StepArgs a;
  memset(&a, 0, sizeof(a));
  a.prm = at<float>(h, h->L.prm);
  a.tiles = nullptr;
  a.fN = at<int>(h, h->L.fN);
  a.fM = at<int>(h, h->L.fM);
  a.ooff = at<int>(h, h->L.ooff);
  a.ioff = at<long long>(h, h->L.ioff);
  a.finfo = at<FilterInfo>(h, h->L.finfo);
  a.ginfo = at<int4>(h, h->L.ginfo);
  a.NT = h->L.NT;
  a.advance = 1;
  a.seed = h->seed;
  a.tcur = at<int>(h, h->L.tcur);
  a.cur = at<unsigned char>(h, h->L.cur);
  a.act = at<unsigned char>(h, h->L.act);
  a.active = nullptr;
  a.run_Tf = nullptr;
  a.run_T = INT_MAX;
  a.x[0] = at<float>(h, h->L.x0);
  a.x[1] = at<float>(h, h->L.x1);
  a.z[0] = at<float>(h, h->L.z0);
  a.z[1] = at<float>(h, h->L.z1);
  a.lam[0] = at<float>(h, h->L.l0);
  a.lam[1] = at<float>(h, h->L.l1);
  a.ell = at<float>(h, h->L.ell);
  a.logw = at<float>(h, h->L.logw);
  a.anc = at<int>(h, h->L.anc);
  a.sel = at<int>(h, h->L.sel);
  a.kpart = at<float>(h, h->L.kpart);
  a.gstat = at<double>(h, h->L.gstat);
  a.fstat = at<double>(h, h->L.fstat);
  a.ess = at<float>(h, h->L.ess);
  a.dlogz = at<double>(h, h->L.dlogz);
  a.loglik = at<double>(h, h->L.loglik);
  a.flags = at<uint32_t>(h, h->L.flags);
  a.est_x = at<float>(h, h->L.est_x);
  a.est_z = at<float>(h, h->L.est_z);
  a.n_filters = h->F;
  a.dy = h->dy;
  a.dx = h->dx;
  a.dz = h->dz;
  a.ind[0] = at<int>(h, h->L.ind0);
  a.ind[1] = at<int>(h, h->L.ind1);
  a.mom = (h->has_proposal && h->eng->moments) ? at<float>(h, h->L.mom) : nullptr;
  a.mlp = at<unsigned char>(h, h->L.mlp);
  a.mdn = at<float>(h, h->L.mdn);
  a.xtmp = at<float>(h, h->L.xtmp);
  a.logq = at<float>(h, h->L.logq);
  a.kpart_tmp = at<float>(h, h->L.kpart_tmp);
  a.mom_tmp = at<float>(h, h->L.mom_tmp);
  a.fb = nullptr;
  a.lflags = at<uint32_t>(h, h->L.lflags);
  a.ess_frac = h->ess_frac;
  a.gpart = at<double>(h, h->L.gpart);
  a.fcount = at<int>(h, h->L.fcount);
  a.n_comp = h->n_comp;
  a.est_y = at<float>(h, h->L.est_y);
  return a;
}

// grid_cap > 0: at most grid_cap workgroups per class, looping over the
// tiles (for launches that most tiles skip).
static dpf_status launch_classes(dpf_handle* h, int op, StepArgs a, int grid_cap = 0) {
  for (const TileClass& tc : h->classes) {
    a.tiles = tc.d_tiles;
    a.n_tiles = tc.n_tiles;
    TileClass g = tc;
    if (grid_cap > 0 && g.n_tiles > grid_cap) g.n_tiles = grid_cap;
    g.n_tiles += a.n_commit;  // extra head workgroups (first class only)
    dpf_status s = h->eng->launch(op, a, g, h->stream);
    a.n_commit = 0;
    if (s != DPF_OK) return s;
  }
  return DPF_OK;
}

constexpr int kGatedGrid = 512;

static dpf_status launch_finalize(dpf_handle* h, const StepArgs& a) {
  return h->eng->finalize(a, h->F, h->stream);
}

// End of a look-ahead step: estimates; next = 1 in a look-ahead run (the
// next step's group statistics, activity and time advance, which spare that
// step its statistics kernel).  Up to kPostFenceGroups groups in the handle:
// one launch whose last workgroup per filter finishes it; more: the group
// pass and a per-filter pass as two launches (same arithmetic).
constexpr int kPostFenceGroups = 64;

static dpf_status launch_post(dpf_handle* h, const StepArgs& a, int next) {
  const int split = h->L.n_rgroups > kPostFenceGroups ? 1 : 0;
  return h->eng->post(a, at<int2>(h, h->L.rgroups), h->L.n_rgroups, h->F, next, split, h->stream);
}

static dpf_status queue_init(dpf_handle* h) {
  h->rb_ready = false;
  const bool plain = h->algo == DPF_ALGO_PLAIN;
  hipLaunchKernelGGL(k_reset, dim3((h->F + 255) / 256), dim3(256), 0, h->stream, at<int>(h, h->L.tcur),
                     at<unsigned char>(h, h->L.cur), at<unsigned char>(h, h->L.act), at<uint32_t>(h, h->L.flags),
                     at<double>(h, h->L.loglik), at<uint32_t>(h, h->L.lflags), at<int>(h, h->L.fcount), h->F);
  LAUNCH_CHECK("k_reset");
  h->mom_valid = false;
  StepArgs a = make_args(h);
  a.advance = 0;
  dpf_status s = launch_classes(h, plain ? OP_INIT_PLAIN : OP_INIT_LA, a);
  // the plain DPF's proposals for t = 1 from the prior (steps 4-7 at t = 0)
  if (s == DPF_OK && plain) s = launch_classes(h, OP_NEWCLOUD_PLAIN, a);
  return s;
}

extern "C" size_t dpf_workspace_bytes(const dpf_config* cfg) {
  const Engine* eng;
  Layout L;
  if (plan(cfg, eng, L) != DPF_OK) return 0;
  return L.total;
}

extern "C" dpf_status dpf_create(const dpf_config* cfg, void* d_workspace, size_t bytes, void* hip_stream,
                                 dpf_handle** out) {
  if (!out) return fail(DPF_EINVAL, "out is NULL");
  *out = nullptr;
  const Engine* eng;
  Layout L;
  dpf_status st = plan(cfg, eng, L);
  if (st != DPF_OK) return st;
  if (!d_workspace) return fail(DPF_EINVAL, "workspace is NULL");
  if (((uintptr_t)d_workspace & 255) != 0) return fail(DPF_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < L.total) return fail(DPF_ENOMEM, "workspace has %zu bytes, needs %zu", bytes, L.total);

  dpf_handle* h = new dpf_handle();
  h->eng = eng;
  h->model = cfg->model;
  h->algo = cfg->algo;
  h->dx = cfg->dx;
  h->dz = cfg->dz;
  h->dy = cfg->dy;
  h->F = cfg->n_filters;
  h->seed = cfg->seed;
  h->stream = (hipStream_t)hip_stream;
  h->L = L;
  h->ws = (char*)d_workspace;
  const int F = h->F;
  h->N.assign(cfg->N, cfg->N + F);
  h->M.assign(cfg->M, cfg->M + F);
  h->ooff.assign(F + 1, 0);
  h->ooff64.assign(F + 1, 0);
  h->ioff.assign(F + 1, 0);
  for (int f = 0; f < F; ++f) {
    h->ooff[f + 1] = h->ooff[f] + h->N[f];
    h->ooff64[f + 1] = h->ooff[f + 1];
    h->ioff[f + 1] = h->ioff[f] + (long long)h->N[f] * h->M[f];
  }
  // parameters: raw values as float, then derived constants
  h->prm_h.reserve(eng->n_total);
  for (size_t q = 0; q < cfg->n_params; ++q) h->prm_h.push_back((float)cfg->params[q]);
  eng->derive(cfg->params, h->prm_h);
  if (h->prm_h.size() != eng->n_total) {
    delete h;
    return fail(DPF_EINVAL, "internal: parameter layout mismatch");
  }
  // per-filter resampling groups; tiles grouped by class (default classes)
  h->finfo_h.assign(F, FilterInfo{0, 0, 0, 0});
  int rg = 0;
  for (int f = 0; f < F; ++f) {
    const int G = (h->N[f] + kResGroup - 1) / kResGroup;
    for (int g = 0; g < G; ++g) {
      h->rgroups_h.push_back(make_int2(f, g));
      h->ginfo_h.push_back(make_int4(h->ooff[f], h->N[f], rg, G));
    }
    h->finfo_h[f] = FilterInfo{rg, G, 0, 0};
    rg += G;
  }
  h->fcls.resize(F);
  for (int f = 0; f < F; ++f) h->fcls[f] = class_of(h->M[f]);
  hipError_t e = hipSuccess;
#define UP(off, vec)                                                                                   \
  if (e == hipSuccess && !(vec).empty())                                                               \
    e = hipMemcpyAsync(h->ws + (off), (vec).data(), (vec).size() * sizeof((vec)[0]), hipMemcpyHostToDevice, \
                       h->stream);
  UP(L.prm, h->prm_h)
  UP(L.fN, h->N)
  UP(L.fM, h->M)
  UP(L.ooff, h->ooff)
  UP(L.ooff64, h->ooff64)
  UP(L.ioff, h->ioff)
  UP(L.rgroups, h->rgroups_h)
  UP(L.ginfo, h->ginfo_h)
  UP(L.finfo, h->finfo_h)
#undef UP
  if (e != hipSuccess) {
    delete h;
    return fail(DPF_EDEVICE, "parameter upload failed: %s", hipGetErrorString(e));
  }
  st = build_tiles(h);
  if (st != DPF_OK) {
    delete h;
    return st;
  }
  st = queue_init(h);
  if (st != DPF_OK) {
    delete h;
    return st;
  }
  *out = h;
  return DPF_OK;
}

// Tiles of every filter in the class h->fcls[f], grouped by class, uploaded
// to the workspace (room for one tile per outer particle was reserved).
static dpf_status build_tiles(dpf_handle* h) {
  const int F = h->F;
  std::vector<std::vector<int4>> by(kNumClasses);
  for (int f = 0; f < F; ++f) {
    const int segs = kBlock / kClasses[h->fcls[f]].seg;
    int nt = 0;
    for (int i0 = 0; i0 < h->N[f]; i0 += segs)
      by[h->fcls[f]].push_back(make_int4(f, i0, nt++, h->finfo_h[f].rg_base));
  }
  h->tiles_h.clear();
  h->classes.clear();
  for (int k = 0; k < kNumClasses; ++k) {
    if (by[k].empty()) continue;
    TileClass tc;
    tc.cls = k;
    tc.n_tiles = (int)by[k].size();
    tc.d_tiles = at<int4>(h, h->L.tiles) + h->tiles_h.size();
    h->tiles_h.insert(h->tiles_h.end(), by[k].begin(), by[k].end());
    h->classes.push_back(tc);
  }
  if ((int)h->tiles_h.size() > h->L.n_tiles) return fail(DPF_EINVAL, "internal: tile room exceeded");
  HIP_TRY(hipMemcpyAsync(h->ws + h->L.tiles, h->tiles_h.data(), h->tiles_h.size() * sizeof(int4),
                         hipMemcpyHostToDevice, h->stream));
  drop_graphs(h);
  return DPF_OK;
}

extern "C" int32_t dpf_tile_classes(int32_t* seg, int32_t* jpt, int32_t n) {
  for (int k = 0; k < kNumClasses && k < n; ++k) {
    if (seg) seg[k] = kClasses[k].seg;
    if (jpt) jpt[k] = kClasses[k].jpt;
  }
  return kNumClasses;
}

extern "C" dpf_status dpf_set_tiling(dpf_handle* h, const int32_t* h_cls) {
  if (!h || !h_cls) return fail(DPF_EINVAL, "handle and class array are required");
  std::vector<int> c(h->F);
  for (int f = 0; f < h->F; ++f) {
    const int k = h_cls[f] < 0 ? class_of(h->M[f]) : h_cls[f];
    if (k >= kNumClasses) return fail(DPF_EINVAL, "class %d of filter %d is not built", k, f);
    if (kClasses[k].seg * kClasses[k].jpt < h->M[f])
      return fail(DPF_EINVAL, "class %d holds %d inner particles, filter %d has M = %d", k,
                  kClasses[k].seg * kClasses[k].jpt, f, h->M[f]);
    c[f] = k;
  }
  h->fcls = c;
  return build_tiles(h);
}

extern "C" dpf_status dpf_reset(dpf_handle* h) {
  if (!h) return fail(DPF_EINVAL, "handle is NULL");
  return queue_init(h);
}

extern "C" dpf_status dpf_destroy(dpf_handle* h) {
  if (!h) return DPF_OK;
  drop_graphs(h);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  delete h;
  return DPF_OK;
}

// fuse (look-ahead runs only): 0 a plain step; 1 the first step of a run,
// whose new-cloud kernel also computes the next step's weights and whose
// step-end kernel also prepares the next step's resampling (group
// statistics, time advance); 2 a later step of the run (no weights or
// statistics kernel: the previous step did their work).  par: the weight
// buffers this step reads (the next step's go to the other pair).
static dpf_status queue_step(dpf_handle* h, const float* Y, long long y_tstride, const unsigned char* active,
                             const int* run_Tf, int run_T, float* trace_x, float* trace_z, int fuse = 0,
                             int par = 0) {
  StepArgs a = make_args(h);
  a.Y = Y;
  a.y_tstride = y_tstride;
  a.active = active;
  a.run_Tf = run_Tf;
  a.run_T = run_T;
  a.trace_x = trace_x;
  a.trace_z = trace_z;
  a.advance = 1;
  const bool plain = h->algo == DPF_ALGO_PLAIN;
  if (fuse) {
    float* e[2] = {at<float>(h, h->L.ell), at<float>(h, h->L.ell1)};
    float* w[2] = {at<float>(h, h->L.logw), at<float>(h, h->L.logw1)};
    a.ell = e[par];
    a.logw = w[par];
    a.ell_next = e[par ^ 1];
    a.logw_next = w[par ^ 1];
  }
  h->ell_sel = fuse ? par : 0;
  if (h->predict && !plain) {
    float* yb[2] = {at<float>(h, h->L.yp0), at<float>(h, h->L.yp1)};
    a.yp = yb[fuse ? par : 0];
    a.yp_next = fuse ? yb[par ^ 1] : nullptr;
    a.trace_y = h->ytrace;
  }
  dpf_status s = phase_mark(h, 0);
  const int wop = plain ? OP_DPF_WEIGHTS : (h->n_comp > 0 ? OP_LA_WEIGHTS_NESTED : OP_LA_WEIGHTS);
  if (s == DPF_OK && fuse != 2) s = launch_classes(h, wop, a);
  if (s == DPF_OK) s = phase_mark(h, 1);
  if (s == DPF_OK && fuse != 2) {
    hipLaunchKernelGGL(k_res_stats, dim3(h->L.n_rgroups), dim3(kBlock), 0, h->stream, a,
                       at<int2>(h, h->L.rgroups), 1);
    LAUNCH_CHECK("k_res_stats");
  }
  if (s == DPF_OK) s = phase_mark(h, 2);
  if (s == DPF_OK) s = launch_classes(h, plain ? OP_NEWCLOUD_PLAIN : OP_NEWCLOUD_LA, a);
  if (s == DPF_OK) s = phase_mark(h, 3);
  if (s == DPF_OK) s = plain ? launch_finalize(h, a) : launch_post(h, a, fuse ? 1 : 0);
  if (s == DPF_OK) s = phase_mark(h, 4);
  h->mom_valid = a.mom != nullptr;
  return s;
}

// Moments of the current state (exact two-pass kernel), for the learned
// step's features; with feat, also the raw feature rows for y.
static dpf_status queue_moments(dpf_handle* h, const float* y, float* feat) {
  if (!h->eng->moments) return fail(DPF_EUNSUPPORTED, "cloud moments are not built for this model");
  StepArgs a = make_args(h);
  a.mom = at<float>(h, h->L.mom);
  g_mom_args = MomArgs{y, feat};
  dpf_status s = launch_classes(h, OP_MOMENTS, a);
  g_mom_args = MomArgs{nullptr, nullptr};
  if (s == DPF_OK) h->mom_valid = true;
  return s;
}

// One learned step (with look-ahead fallback per filter); mdn_given: the
// network outputs [NT][32] supplied by the caller instead of the network.
static dpf_status queue_learned_step(dpf_handle* h, const float* Y, long long y_tstride,
                                     const unsigned char* active, const int* run_Tf, int run_T, float* trace_x,
                                     float* trace_z, const float* mdn_given) {
  h->rb_ready = false;
  dpf_status s = DPF_OK;
  if (!h->mom_valid && !mdn_given) s = queue_moments(h, nullptr, nullptr);
  if (s != DPF_OK) return s;
  h->ell_sel = 0;
  StepArgs a = make_args(h);
  a.Y = Y;
  a.y_tstride = y_tstride;
  a.active = active;
  a.run_Tf = run_Tf;
  a.run_T = run_T;
  a.trace_x = trace_x;
  a.trace_z = trace_z;
  a.advance = 1;
  a.mom = at<float>(h, h->L.mom);
  if (mdn_given) a.mdn = const_cast<float*>(mdn_given);
  s = phase_mark(h, 0);
  if (s == DPF_OK) s = mdn_given ? h->eng->mdn_draw(a, h->stream) : h->eng->mlp_state(a, h->stream);
  if (s == DPF_OK) s = launch_classes(h, OP_LEARNED_INNER, a);
  if (s == DPF_OK) s = phase_mark(h, 1);
  if (s == DPF_OK) {
    hipLaunchKernelGGL(k_res_stats, dim3(h->L.n_rgroups), dim3(kBlock), 0, h->stream, a,
                       at<int2>(h, h->L.rgroups), 0);
    LAUNCH_CHECK("k_res_stats");
  }
  a.fb = at<unsigned char>(h, h->L.fb);
  if (s == DPF_OK) s = launch_classes(h, OP_LA_WEIGHTS_FALLBACK, a, kGatedGrid);
  if (s == DPF_OK) {
    hipLaunchKernelGGL(k_res_stats, dim3(h->L.n_rgroups), dim3(kBlock), 0, h->stream, a,
                       at<int2>(h, h->L.rgroups), 1);
    LAUNCH_CHECK("k_res_stats");
  }
  if (s == DPF_OK) s = phase_mark(h, 2);
  // one launch per class: the commit of accepted filters (first class) and the
  // look-ahead new clouds of the filters that fell back
  a.rgroups = at<int2>(h, h->L.rgroups);
  a.n_commit = h->L.n_rgroups;
  if (s == DPF_OK) s = launch_classes(h, OP_NEWCLOUD_FALLBACK, a, kGatedGrid);
  if (s == DPF_OK) s = phase_mark(h, 3);
  if (s == DPF_OK) s = launch_post(h, a, 0);
  if (s == DPF_OK) s = phase_mark(h, 4);
  h->mom_valid = true;
  return s;
}

extern "C" dpf_status dpf_set_phase_events(dpf_handle* h, void* const* hip_events, int32_t n_events) {
  if (!h) return fail(DPF_EINVAL, "handle is NULL");
  if (n_events < 0 || (n_events > 0 && !hip_events)) return fail(DPF_EINVAL, "bad event array");
  if (n_events % kPhaseEvents) return fail(DPF_EINVAL, "n_events must be a multiple of %d", kPhaseEvents);
  h->prof_events.assign((hipEvent_t*)hip_events, (hipEvent_t*)hip_events + n_events);
  h->prof_next = 0;
  return DPF_OK;
}

extern "C" dpf_status dpf_lookahead_step(dpf_handle* h, const float* d_y, const uint8_t* d_active) {
  if (!h || !d_y) return fail(DPF_EINVAL, "handle and d_y are required");
  if (h->algo != DPF_ALGO_LOOKAHEAD) return fail(DPF_ESTATE, "handle was created for the plain DPF");
  h->rb_ready = false;
  const dpf_status s = queue_step(h, d_y, 0, d_active, nullptr, INT_MAX, nullptr, nullptr);
  h->rb_ready = s == DPF_OK;
  return s;
}

extern "C" dpf_status dpf_set_lookahead_companions(dpf_handle* h, int32_t n_comp) {
  if (!h) return fail(DPF_EINVAL, "handle is NULL");
  if (h->algo != DPF_ALGO_LOOKAHEAD) return fail(DPF_ESTATE, "companions belong to the look-ahead DPF");
  if (n_comp < 0 || n_comp > kMaxCompanions)
    return fail(DPF_EINVAL, "n_comp = %d outside 0..%d", n_comp, kMaxCompanions);
  h->n_comp = n_comp;
  return DPF_OK;
}

extern "C" dpf_status dpf_set_prediction(dpf_handle* h, int32_t enable, float* d_ytrace) {
  if (!h) return fail(DPF_EINVAL, "handle is NULL");
  if (h->algo != DPF_ALGO_LOOKAHEAD) return fail(DPF_ESTATE, "the prediction is formed by the look-ahead pass");
  if (enable && !h->eng->yhat)
    return fail(DPF_EUNSUPPORTED, "model %d has no built predicted observation (one-dimensional y only)", h->model);
  h->predict = enable != 0;
  h->ytrace = enable ? d_ytrace : nullptr;
  return DPF_OK;
}

extern "C" dpf_status dpf_predicted_observation(dpf_handle* h, float* d_yhat) {
  if (!h || !d_yhat) return fail(DPF_EINVAL, "handle and d_yhat are required");
  if (!h->predict) return fail(DPF_ESTATE, "prediction is not enabled (dpf_set_prediction)");
  HIP_TRY(hipMemcpyAsync(d_yhat, h->ws + h->L.est_y, (size_t)h->F * 4, hipMemcpyDeviceToDevice, h->stream));
  return DPF_OK;
}

extern "C" dpf_status dpf_estimate_rb(dpf_handle* h, float* d_xrb) {
  if (!h || !d_xrb) return fail(DPF_EINVAL, "handle and d_xrb are required");
  if (!h->rb_ready) return fail(DPF_ESTATE, "dpf_estimate_rb follows a dpf_lookahead_step call");
  StepArgs a = make_args(h);
  a.ell = at<float>(h, h->ell_sel ? h->L.ell1 : h->L.ell);
  a.logw = at<float>(h, h->ell_sel ? h->L.logw1 : h->L.logw);
  return h->eng->rb(a, at<double>(h, h->L.xrb), d_xrb, h->stream);
}

extern "C" dpf_status dpf_step(dpf_handle* h, const float* d_y, const uint8_t* d_active) {
  if (!h || !d_y) return fail(DPF_EINVAL, "handle and d_y are required");
  if (h->algo != DPF_ALGO_PLAIN) return fail(DPF_ESTATE, "handle was created for the look-ahead DPF");
  return queue_step(h, d_y, 0, d_active, nullptr, INT_MAX, nullptr, nullptr);
}

static dpf_status check_learned(dpf_handle* h) {
  if (h->algo != DPF_ALGO_LOOKAHEAD) return fail(DPF_ESTATE, "the learned step needs a look-ahead handle");
  if (!h->eng->mlp_state) return fail(DPF_EUNSUPPORTED, "no learned proposal for model %d", h->model);
  return DPF_OK;
}

extern "C" dpf_status dpf_set_proposal(dpf_handle* h, const void* d_blob, size_t bytes, double ess_frac) {
  if (!h || !d_blob) return fail(DPF_EINVAL, "handle and blob are required");
  dpf_status s = check_learned(h);
  if (s != DPF_OK) return s;
  if (bytes != MlpBlobLayout::bytes) return fail(DPF_EINVAL, "blob has %zu bytes, expected %zu", bytes,
                                                 (size_t)MlpBlobLayout::bytes);
  if (!(ess_frac >= 0.0 && ess_frac <= 1.0)) return fail(DPF_EINVAL, "ess_frac must lie in [0, 1]");
  HIP_TRY(hipMemcpyAsync(h->ws + h->L.mlp, d_blob, bytes, hipMemcpyDeviceToDevice, h->stream));
  h->has_proposal = true;
  h->ess_frac = ess_frac;
  return queue_moments(h, nullptr, nullptr);
}

extern "C" dpf_status dpf_learned_step(dpf_handle* h, const float* d_y, const uint8_t* d_active) {
  if (!h || !d_y) return fail(DPF_EINVAL, "handle and d_y are required");
  dpf_status s = check_learned(h);
  if (s != DPF_OK) return s;
  if (!h->has_proposal) return fail(DPF_ESTATE, "no proposal set (dpf_set_proposal)");
  return queue_learned_step(h, d_y, 0, d_active, nullptr, INT_MAX, nullptr, nullptr, nullptr);
}

extern "C" dpf_status dpf_learned_step_given(dpf_handle* h, const float* d_y, const uint8_t* d_active,
                                             const float* d_mdn, double ess_frac) {
  if (!h || !d_y || !d_mdn) return fail(DPF_EINVAL, "handle, d_y and d_mdn are required");
  dpf_status s = check_learned(h);
  if (s != DPF_OK) return s;
  if (!(ess_frac >= 0.0 && ess_frac <= 1.0)) return fail(DPF_EINVAL, "ess_frac must lie in [0, 1]");
  const double keep = h->ess_frac;
  h->ess_frac = ess_frac;
  s = queue_learned_step(h, d_y, 0, d_active, nullptr, INT_MAX, nullptr, nullptr, d_mdn);
  h->ess_frac = keep;
  return s;
}

extern "C" dpf_status dpf_features(dpf_handle* h, const float* d_y, float* d_feat) {
  if (!h || !d_y || !d_feat) return fail(DPF_EINVAL, "handle, d_y and d_feat are required");
  dpf_status s = check_learned(h);
  if (s != DPF_OK) return s;
  return queue_moments(h, d_y, d_feat);
}

extern "C" dpf_status dpf_estimate(dpf_handle* h, float* d_xmean, float* d_zmean, float* d_ess,
                                   double* d_loglik, uint32_t* d_flags) {
  if (!h) return fail(DPF_EINVAL, "handle is NULL");
  const int F = h->F;
  if (d_xmean)
    HIP_TRY(hipMemcpyAsync(d_xmean, h->ws + h->L.est_x, (size_t)F * h->dx * 4, hipMemcpyDeviceToDevice, h->stream));
  if (d_zmean)
    HIP_TRY(hipMemcpyAsync(d_zmean, h->ws + h->L.est_z, (size_t)F * h->dz * 4, hipMemcpyDeviceToDevice, h->stream));
  if (d_ess) HIP_TRY(hipMemcpyAsync(d_ess, h->ws + h->L.ess, (size_t)F * 4, hipMemcpyDeviceToDevice, h->stream));
  if (d_loglik)
    HIP_TRY(hipMemcpyAsync(d_loglik, h->ws + h->L.loglik, (size_t)F * 8, hipMemcpyDeviceToDevice, h->stream));
  if (d_flags)
    HIP_TRY(hipMemcpyAsync(d_flags, h->ws + h->L.flags, (size_t)F * 4, hipMemcpyDeviceToDevice, h->stream));
  return DPF_OK;
}

// Step q (0-based) of a run; look-ahead runs fuse the weights of each step
// into the previous step's new-cloud kernel.
static dpf_status queue_run_step(dpf_handle* h, int mode, const float* d_Y, int T, const int32_t* d_Tf,
                                 float* xt, float* zt, int q) {
  const long long stride = (long long)h->F * h->dy;
  if (mode == 1) return queue_learned_step(h, d_Y, stride, nullptr, (const int*)d_Tf, T, xt, zt, nullptr);
  // (the fused next-step weights are the paired form: a nested run takes
  // every step whole)
  if (h->algo == DPF_ALGO_LOOKAHEAD && T > 1 && h->n_comp == 0)
    return queue_step(h, d_Y, stride, nullptr, (const int*)d_Tf, T, xt, zt, q == 0 ? 1 : 2, q & 1);
  return queue_step(h, d_Y, stride, nullptr, (const int*)d_Tf, T, xt, zt);
}

// T steps of mode 0 (the handle's algorithm) or 1 (learned), eagerly or as
// replays of a captured chunk of S = min(T - 1, kGraphChunk) steps (every
// step reads the per-filter time and state copy from device memory, so one
// capture serves every chunk), the last (T - 1) mod S steps as a second
// captured graph.  The first step always runs eagerly (in a look-ahead run it
// is the only one with a weights kernel); kGraphChunk is even, so repeated
// chunks and the tail see the same alternation of weight buffers.  Each graph
// launch costs a gap of several microseconds between the kernels of
// successive steps, hence long chunks.
constexpr int kGraphChunk = 256;

static dpf_status run_steps(dpf_handle* h, int mode, const float* d_Y, int32_t T, const int32_t* d_Tf,
                            float* d_xtrace, float* d_ztrace, int32_t use_graph) {
  if (!h || !d_Y) return fail(DPF_EINVAL, "handle and d_Y are required");
  if (T < 0) return fail(DPF_EINVAL, "T = %d", T);
  h->rb_ready = false;
  if (T == 0) return DPF_OK;
  if (mode == 1 && !h->mom_valid) {
    // moments of the starting state, outside any captured step
    dpf_status st = queue_moments(h, nullptr, nullptr);
    if (st != DPF_OK) return st;
  }
  if (!use_graph) {
    for (int s = 0; s < T; ++s) {
      dpf_status st = queue_run_step(h, mode, d_Y, T, d_Tf, d_xtrace, d_ztrace, s);
      if (st != DPF_OK) return st;
    }
    return DPF_OK;
  }
  {
    dpf_status st = queue_run_step(h, mode, d_Y, T, d_Tf, d_xtrace, d_ztrace, 0);
    if (st != DPF_OK || T == 1) return st;
  }
  const int S = T - 1 < kGraphChunk ? T - 1 : kGraphChunk;
  const int R = (T - 1) % S;  // tail steps T - R .. T - 1
  // every value make_args copies into the captured kernel arguments that can
  // change between runs is part of the key: the buffers, the stream, the
  // mode, whether cloud moments are maintained, and the fallback threshold
  uint64_t ess_bits;
  memcpy(&ess_bits, &h->ess_frac, sizeof(ess_bits));
  const void* key[11] = {d_Y, d_Tf, d_xtrace, d_ztrace, (const void*)h->stream, (const void*)(intptr_t)mode,
                         (const void*)(intptr_t)(h->has_proposal ? 1 : 0), (const void*)(uintptr_t)ess_bits,
                         (const void*)(intptr_t)h->n_comp, (const void*)(intptr_t)(h->predict ? 1 : 0),
                         (const void*)h->ytrace};
  const bool cached = h->gexec && h->g_T == T && memcmp(key, h->g_key, sizeof(key)) == 0;
  if (!cached) {
    drop_graphs(h);
    if (!h->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    // steps q0 .. q0 + n - 1 captured into *out
    auto capture = [&](int q0, int n, hipGraphExec_t* out) -> dpf_status {
      hipStream_t user = h->stream;
      h->stream = h->cap_stream;
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal);
      dpf_status st = DPF_OK;
      for (int q = q0; e == hipSuccess && st == DPF_OK && q < q0 + n; ++q)
        st = queue_run_step(h, mode, d_Y, T, d_Tf, d_xtrace, d_ztrace, q);
      hipError_t e2 = hipStreamEndCapture(h->cap_stream, &g);
      h->stream = user;
      if (e != hipSuccess) return fail(DPF_EDEVICE, "hipStreamBeginCapture: %s", hipGetErrorString(e));
      if (st != DPF_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
      }
      if (e2 != hipSuccess) return fail(DPF_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e2));
      e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) {
        *out = nullptr;
        return fail(DPF_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
      }
      return DPF_OK;
    };
    dpf_status st = capture(1, S, &h->gexec);
    if (st == DPF_OK && R > 0) st = capture(T - R, R, &h->gexec_tail);
    if (st != DPF_OK) {
      drop_graphs(h);
      return st;
    }
    memcpy(h->g_key, key, sizeof(key));
    h->g_T = T;
  }
  for (int q = 1; q + S <= T; q += S) HIP_TRY(hipGraphLaunch(h->gexec, h->stream));
  if (R > 0) HIP_TRY(hipGraphLaunch(h->gexec_tail, h->stream));
  // (the captured steps do not update the host's record of the buffers)
  if (mode == 0 && h->algo == DPF_ALGO_LOOKAHEAD && h->n_comp == 0) h->ell_sel = (T - 1) & 1;
  return DPF_OK;
}

extern "C" dpf_status dpf_run(dpf_handle* h, const float* d_Y, int32_t T, const int32_t* d_Tf, float* d_xtrace,
                              float* d_ztrace, int32_t use_graph) {
  return run_steps(h, 0, d_Y, T, d_Tf, d_xtrace, d_ztrace, use_graph);
}

extern "C" dpf_status dpf_learned_run(dpf_handle* h, const float* d_Y, int32_t T, const int32_t* d_Tf,
                                      float* d_xtrace, float* d_ztrace, int32_t use_graph) {
  if (!h) return fail(DPF_EINVAL, "handle is NULL");
  dpf_status s = check_learned(h);
  if (s != DPF_OK) return s;
  if (!h->has_proposal) return fail(DPF_ESTATE, "no proposal set (dpf_set_proposal)");
  return run_steps(h, 1, d_Y, T, d_Tf, d_xtrace, d_ztrace, use_graph);
}

// ---------------------------------------------------------------- state I/O
static size_t state_time_bytes(int F) { return ((size_t)F * 4 + 15) & ~(size_t)15; }

extern "C" size_t dpf_state_bytes(const dpf_handle* h) {
  if (!h) return 0;
  return state_time_bytes(h->F) + (size_t)h->L.NT * h->dx * 4 + (size_t)h->L.NMT * h->dz * 4 +
         (size_t)h->L.NMT * 4;
}

static dpf_status state_io(dpf_handle* h, char* ext, int dir) {
  if (dir == 1) h->rb_ready = false;
  const int F = h->F;
  const size_t tb = state_time_bytes(F);
  float* ex = (float*)(ext + tb);
  float* ez = ex + (size_t)h->L.NT * h->dx;
  float* el = ez + (size_t)h->L.NMT * h->dz;
  const unsigned char* cur = at<unsigned char>(h, h->L.cur);
  const long long* ioff = at<long long>(h, h->L.ioff);
  const long long* oo64 = at<long long>(h, h->L.ooff64);
  const int B = 256;
  const long long nx = (long long)h->L.NT * h->dx, nz = h->L.NMT * h->dz, nl = h->L.NMT;
  if (dir == 0) {
    const int words = (int)(tb / 4);
    hipLaunchKernelGGL(k_export_time, dim3((words + 255) / 256), dim3(256), 0, h->stream, at<int>(h, h->L.tcur),
                       (int*)ext, F, words);
    LAUNCH_CHECK("k_export_time");
  }
  hipLaunchKernelGGL(k_state_copy_x, dim3((unsigned)((nx + B - 1) / B)), dim3(B), 0, h->stream, ex,
                     at<float>(h, h->L.x0), at<float>(h, h->L.x1), cur, oo64, F, h->L.NT, h->dx, dir);
  if (h->algo == DPF_ALGO_LOOKAHEAD) {
    const int* i0 = at<int>(h, h->L.ind0);
    const int* i1 = at<int>(h, h->L.ind1);
    const int* oo = at<int>(h, h->L.ooff);
    const int* fm = at<int>(h, h->L.fM);
    hipLaunchKernelGGL(k_state_copy_cloud, dim3((unsigned)((nz + B - 1) / B)), dim3(B), 0, h->stream, ez,
                       at<float>(h, h->L.z0), at<float>(h, h->L.z1), i0, i1, cur, ioff, oo, fm, F,
                       h->L.NMT, h->dz, dir);
    hipLaunchKernelGGL(k_state_copy_cloud, dim3((unsigned)((nl + B - 1) / B)), dim3(B), 0, h->stream, el,
                       at<float>(h, h->L.l0), at<float>(h, h->L.l1), i0, i1, cur, ioff, oo, fm, F,
                       h->L.NMT, 1, dir);
  } else {
    hipLaunchKernelGGL(k_state_copy, dim3((unsigned)((nz + B - 1) / B)), dim3(B), 0, h->stream, ez,
                       at<float>(h, h->L.z0), at<float>(h, h->L.z1), cur, ioff, F, h->L.NMT, h->dz, dir);
    hipLaunchKernelGGL(k_state_copy, dim3((unsigned)((nl + B - 1) / B)), dim3(B), 0, h->stream, el,
                       at<float>(h, h->L.l0), at<float>(h, h->L.l1), cur, ioff, F, h->L.NMT, 1, dir);
  }
  LAUNCH_CHECK("state copy");
  if (dir == 1) h->mom_valid = false;
  if (dir == 1) {
    hipLaunchKernelGGL(k_import_time, dim3((F + 255) / 256), dim3(256), 0, h->stream, (const int*)ext,
                       at<int>(h, h->L.tcur), at<unsigned char>(h, h->L.cur), at<uint32_t>(h, h->L.flags),
                       at<double>(h, h->L.loglik), F);
    LAUNCH_CHECK("k_import_time");
  }
  return DPF_OK;
}

extern "C" dpf_status dpf_export_state(dpf_handle* h, void* d_dst, size_t bytes) {
  if (!h || !d_dst) return fail(DPF_EINVAL, "handle and destination are required");
  if (bytes < dpf_state_bytes(h)) return fail(DPF_EINVAL, "state needs %zu bytes", dpf_state_bytes(h));
  return state_io(h, (char*)d_dst, 0);
}

extern "C" dpf_status dpf_import_state(dpf_handle* h, const void* d_src, size_t bytes) {
  if (!h || !d_src) return fail(DPF_EINVAL, "handle and source are required");
  if (bytes < dpf_state_bytes(h)) return fail(DPF_EINVAL, "state needs %zu bytes", dpf_state_bytes(h));
  return state_io(h, (char*)d_src, 1);
}

extern "C" dpf_status dpf_copy_buffer(dpf_handle* h, int32_t which, void* d_dst, size_t bytes) {
  if (!h || !d_dst) return fail(DPF_EINVAL, "handle and destination are required");
  size_t off = 0, need = 0;
  switch (which) {
    case DPF_BUF_ELL: off = h->ell_sel ? h->L.ell1 : h->L.ell; need = (size_t)h->L.NMT * 4; break;
    case DPF_BUF_LOGW: off = h->ell_sel ? h->L.logw1 : h->L.logw; need = (size_t)h->L.NT * 4; break;
    case DPF_BUF_ANC: off = h->L.anc; need = (size_t)h->L.NT * 4; break;
    case DPF_BUF_SEL: off = h->L.sel; need = (size_t)h->L.NT * 4; break;
    case DPF_BUF_MDN: off = h->L.mdn; need = (size_t)h->L.NT * kMlpOut * 4; break;
    case DPF_BUF_FALLBACK: off = h->L.fb; need = (size_t)h->F; break;
    case DPF_BUF_X: {
      need = (size_t)h->L.NT * h->dx * 4;
      if (bytes < need) return fail(DPF_EINVAL, "buffer %d needs %zu bytes", which, need);
      const long long nx = (long long)h->L.NT * h->dx;
      hipLaunchKernelGGL(k_state_copy_x, dim3((unsigned)((nx + 255) / 256)), dim3(256), 0, h->stream,
                         (float*)d_dst, at<float>(h, h->L.x0), at<float>(h, h->L.x1),
                         at<unsigned char>(h, h->L.cur), at<long long>(h, h->L.ooff64), h->F, h->L.NT, h->dx, 0);
      LAUNCH_CHECK("k_state_copy_x");
      return DPF_OK;
    }
    default: return fail(DPF_EINVAL, "unknown buffer %d", which);
  }
  if (bytes < need) return fail(DPF_EINVAL, "buffer %d needs %zu bytes", which, need);
  HIP_TRY(hipMemcpyAsync(d_dst, h->ws + off, need, hipMemcpyDeviceToDevice, h->stream));
  return DPF_OK;
}

// ---------------------------------------------------------------- primitives
extern "C" dpf_status dpf_philox_words(uint64_t seed, uint32_t filter_id, const uint32_t* d_ctr, size_t n,
                                       uint32_t* d_out, void* hip_stream) {
  if ((!d_ctr || !d_out) && n) return fail(DPF_EINVAL, "null buffer");
  if (n == 0) return DPF_OK;
  hipLaunchKernelGGL(k_philox_words, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)hip_stream,
                     make_key(seed, filter_id), d_ctr, (long long)n, d_out);
  LAUNCH_CHECK("k_philox_words");
  return DPF_OK;
}

extern "C" dpf_status dpf_normals(uint64_t seed, uint32_t filter_id, uint32_t t, uint32_t purpose, int32_t n_a,
                                  int32_t n_b, int32_t D, float* d_out, void* hip_stream) {
  if (!d_out || n_a < 0 || n_b < 0) return fail(DPF_EINVAL, "bad arguments");
  const long long n = (long long)n_a * n_b;
  if (n == 0) return DPF_OK;
  const dim3 g((unsigned)((n + 255) / 256));
  const Key key = make_key(seed, filter_id);
  hipStream_t s = (hipStream_t)hip_stream;
  switch (D) {
    case 1: hipLaunchKernelGGL(k_normals_grid<1>, g, dim3(256), 0, s, key, t, purpose, n_a, n_b, d_out); break;
    case 2: hipLaunchKernelGGL(k_normals_grid<2>, g, dim3(256), 0, s, key, t, purpose, n_a, n_b, d_out); break;
    case 4: hipLaunchKernelGGL(k_normals_grid<4>, g, dim3(256), 0, s, key, t, purpose, n_a, n_b, d_out); break;
    case 8: hipLaunchKernelGGL(k_normals_grid<8>, g, dim3(256), 0, s, key, t, purpose, n_a, n_b, d_out); break;
    case 10: hipLaunchKernelGGL(k_normals_grid<10>, g, dim3(256), 0, s, key, t, purpose, n_a, n_b, d_out); break;
    case 64: hipLaunchKernelGGL(k_normals_grid<64>, g, dim3(256), 0, s, key, t, purpose, n_a, n_b, d_out); break;
    case 68: hipLaunchKernelGGL(k_normals_grid<68>, g, dim3(256), 0, s, key, t, purpose, n_a, n_b, d_out); break;
    default: return fail(DPF_EUNSUPPORTED, "D = %d (built: 1, 2, 4, 8, 10, 64, 68)", D);
  }
  LAUNCH_CHECK("k_normals_grid");
  return DPF_OK;
}

extern "C" dpf_status dpf_systematic(const double* d_w, int32_t n, int32_t n_out, double u, double* d_scratch,
                                     int32_t* d_out, void* hip_stream) {
  if (!d_w || !d_out || !d_scratch || n < 1 || n_out < 1) return fail(DPF_EINVAL, "bad arguments");
  if (n > 65536) return fail(DPF_EUNSUPPORTED, "n = %d > 65536", n);
  if (!(u >= 0.0 && u < 1.0)) return fail(DPF_EINVAL, "u must be in [0, 1)");
  const int G = (n + kResGroup - 1) / kResGroup;
  hipStream_t s = (hipStream_t)hip_stream;
  hipLaunchKernelGGL(k_prim_res_stats, dim3(G), dim3(kBlock), 0, s, d_w, n, d_scratch);
  LAUNCH_CHECK("k_prim_res_stats");
  hipLaunchKernelGGL(k_prim_res_select, dim3((n_out + kBlock - 1) / kBlock), dim3(kBlock), 0, s, d_w, n, n_out, u,
                     d_scratch, (int*)d_out);
  LAUNCH_CHECK("k_prim_res_select");
  return DPF_OK;
}

// ------------------------------------------------ systematic, no allocation
// dpf_systematic_noalloc keeps the per-group statistics in this file-scope
// device array instead of a caller-supplied scratch buffer.  In host code
// the name is only a stand-in: kernels get the address that
// hipGetSymbolAddress returns for the current device (each device holds its
// own copy), looked up once per device on the first call there.
constexpr int kNoAllocMaxN = 65536;
constexpr int kNoAllocGroups = kNoAllocMaxN / kResGroup;
static __device__ __align__(256) double scratch[4 * kNoAllocGroups];
constexpr int kMaxDevices = 64;
static double* g_scratch_dev[kMaxDevices];
static std::mutex g_scratch_mu;

static dpf_status scratch_for_current_device(double** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(DPF_EUNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    double* p = nullptr;
    const hipError_t e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(DPF_EDEVICE, "hipGetSymbolAddress of the scratch array failed: %s", hipGetErrorString(e));
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return DPF_OK;
}

extern "C" dpf_status dpf_systematic_noalloc(const double* d_w, int32_t n, int32_t n_out, double u, int32_t* d_out,
                                             void* hip_stream) {
  if (!d_w || !d_out || n < 1 || n_out < 1) return fail(DPF_EINVAL, "bad arguments");
  if (n > kNoAllocMaxN)
    return fail(DPF_EUNSUPPORTED, "n = %d exceeds the %d weights the library's own scratch holds", n, kNoAllocMaxN);
  if (!(u >= 0.0 && u < 1.0)) return fail(DPF_EINVAL, "u must be in [0, 1)");
  double* ws = nullptr;
  const dpf_status st = scratch_for_current_device(&ws);
  if (st != DPF_OK) return st;
  // every group entry the kernels read is written by the statistics launch
  // of this call first, so nothing needs clearing
  const int G = (n + kResGroup - 1) / kResGroup;
  hipStream_t s = (hipStream_t)hip_stream;
  hipLaunchKernelGGL(k_prim_res_stats, dim3(G), dim3(kBlock), 0, s, d_w, n, ws);
  LAUNCH_CHECK("k_prim_res_stats");
  hipLaunchKernelGGL(k_prim_res_select, dim3((n_out + kBlock - 1) / kBlock), dim3(kBlock), 0, s, d_w, n, n_out, u,
                     (const double*)ws, (int*)d_out);
  LAUNCH_CHECK("k_prim_res_select");
  return DPF_OK;
}

extern "C" dpf_status dpf_segmented_systematic(const double* d_w, int32_t S, int32_t n, int32_t n_out,
                                               const double* d_u, int32_t* d_out, void* hip_stream) {
  if (!d_w || !d_u || !d_out || S < 0 || n < 1) return fail(DPF_EINVAL, "bad arguments");
  if (n_out != n && n_out != 1) return fail(DPF_EINVAL, "n_out must be n or 1");
  if (S == 0) return DPF_OK;
  const int cls = class_of(n);
  if (cls < 0) return fail(DPF_EUNSUPPORTED, "n = %d > 4096", n);
  const int segs = kBlock / kClasses[cls].seg;
  const dim3 g((S + segs - 1) / segs);
  hipStream_t s = (hipStream_t)hip_stream;
  switch (cls) {
    case 0: hipLaunchKernelGGL((k_seg_systematic_prim<32, 1>), g, dim3(kBlock), 0, s, d_w, S, n, n_out, d_u, (int*)d_out); break;
    case 1: hipLaunchKernelGGL((k_seg_systematic_prim<64, 1>), g, dim3(kBlock), 0, s, d_w, S, n, n_out, d_u, (int*)d_out); break;
    case 2: hipLaunchKernelGGL((k_seg_systematic_prim<128, 1>), g, dim3(kBlock), 0, s, d_w, S, n, n_out, d_u, (int*)d_out); break;
    case 3: hipLaunchKernelGGL((k_seg_systematic_prim<64, 4>), g, dim3(kBlock), 0, s, d_w, S, n, n_out, d_u, (int*)d_out); break;
    case 4: hipLaunchKernelGGL((k_seg_systematic_prim<256, 4>), g, dim3(kBlock), 0, s, d_w, S, n, n_out, d_u, (int*)d_out); break;
    case 5: hipLaunchKernelGGL((k_seg_systematic_prim<256, 16>), g, dim3(kBlock), 0, s, d_w, S, n, n_out, d_u, (int*)d_out); break;
  }
  LAUNCH_CHECK("k_seg_systematic_prim");
  return DPF_OK;
}

// ---------------------------------------------------------------- network
// Training workspace (batch B, a multiple of 32): the transposed BF16
// weights first (fixed offsets, written by dpf_mlp_pack and the Adam
// kernel), then the activations, gradients and partial sums of one step.
struct TrainWs {
  size_t w2t, w3t, out, a1, a2, x0t, h1t, h2t, gb, gt, da2t, da1t, wp1, wp2, wp3, b1p, b2p, b3p, lossp, total;
  int chunks, tiles, groups;
};

static TrainWs train_layout(int B) {
  TrainWs w;
  size_t c = 0;
  w.chunks = (B + kWgChunk - 1) / kWgChunk;
  w.tiles = (B + kMlpRows - 1) / kMlpRows;
  w.groups = (B + kBlock - 1) / kBlock;
  const size_t b = (size_t)B;
  w.w2t = carve(c, (size_t)kMlpHid * kMlpHid * 2);
  w.w3t = carve(c, (size_t)kMlpHid * kMlpOut * 2);
  w.out = carve(c, b * kMlpOut * 4);
  w.a1 = carve(c, b * kMlpHid * 4);
  w.a2 = carve(c, b * kMlpHid * 4);
  w.x0t = carve(c, b * kMlpIn * 2);
  w.h1t = carve(c, b * kMlpHid * 2);
  w.h2t = carve(c, b * kMlpHid * 2);
  w.gb = carve(c, b * kMlpOut * 2);
  w.gt = carve(c, b * kMlpOut * 2);
  w.da2t = carve(c, b * kMlpHid * 2);
  w.da1t = carve(c, b * kMlpHid * 2);
  w.wp1 = carve(c, (size_t)w.chunks * kMlpHid * kMlpIn * 4);
  w.wp2 = carve(c, (size_t)w.chunks * kMlpHid * kMlpHid * 4);
  w.wp3 = carve(c, (size_t)w.chunks * kMlpOut * kMlpHid * 4);
  w.b1p = carve(c, (size_t)w.tiles * kMlpHid * 4);
  w.b2p = carve(c, (size_t)w.tiles * kMlpHid * 4);
  w.b3p = carve(c, (size_t)w.groups * kMlpOut * 4);
  w.lossp = carve(c, (size_t)w.groups * 8);
  w.total = c;
  return w;
}

constexpr int kMaxTrainBatch = 1 << 20;

extern "C" size_t dpf_mlp_blob_bytes(void) { return MlpBlobLayout::bytes; }
extern "C" size_t dpf_mlp_param_count(void) { return MlpParamLayout::n; }

extern "C" size_t dpf_mlp_train_workspace_bytes(int32_t batch) {
  if (batch < 32 || batch % 32 != 0 || batch > kMaxTrainBatch) return 0;
  return train_layout(batch).total;
}

extern "C" dpf_status dpf_mlp_pack(const float* d_params, const float* d_fmean, const float* d_fstd, void* d_blob,
                                   void* d_train_ws, size_t ws_bytes, void* hip_stream) {
  if (!d_params || !d_fmean || !d_fstd || !d_blob) return fail(DPF_EINVAL, "params, fmean, fstd and blob are required");
  const TrainWs w = train_layout(32);
  if (d_train_ws && ws_bytes < w.w3t + (size_t)kMlpHid * kMlpOut * 2)
    return fail(DPF_EINVAL, "training workspace too small");
  char* ws = (char*)d_train_ws;
  hipLaunchKernelGGL(k_mlp_pack, dim3((MlpParamLayout::n + 255) / 256), dim3(256), 0, (hipStream_t)hip_stream,
                     d_params, d_fmean, d_fstd, (unsigned char*)d_blob, ws ? (bf16_t*)(ws + w.w2t) : nullptr,
                     ws ? (bf16_t*)(ws + w.w3t) : nullptr);
  LAUNCH_CHECK("k_mlp_pack");
  return DPF_OK;
}

extern "C" dpf_status dpf_mlp_forward(const void* d_blob, const float* d_X, int32_t B, float* d_out,
                                      void* hip_stream) {
  if (!d_blob || (!d_X && B) || (!d_out && B) || B < 0) return fail(DPF_EINVAL, "bad arguments");
  if (B == 0) return DPF_OK;
  hipLaunchKernelGGL(k_mlp_fwd_x<false>, dim3((B + kMlpRows - 1) / kMlpRows), dim3(kBlock), 0,
                     (hipStream_t)hip_stream, (const unsigned char*)d_blob, d_X, B, d_out, MlpTrainOut{});
  LAUNCH_CHECK("k_mlp_fwd_x");
  return DPF_OK;
}

extern "C" dpf_status dpf_mlp_train_step(float* d_state, void* d_blob, const float* d_X, const float* d_xt,
                                         int32_t B, float lr, int32_t adam_t, void* d_train_ws, size_t ws_bytes,
                                         float* d_loss, float* d_grad, void* hip_stream) {
  if (!d_state || !d_blob || !d_X || !d_xt || !d_train_ws) return fail(DPF_EINVAL, "null buffer");
  if (B < 32 || B % 32 != 0 || B > kMaxTrainBatch)
    return fail(DPF_EINVAL, "batch %d must be a positive multiple of 32 up to %d", B, kMaxTrainBatch);
  if (adam_t < 0) return fail(DPF_EINVAL, "adam_t = %d", adam_t);
  const TrainWs w = train_layout(B);
  if (ws_bytes < w.total) return fail(DPF_EINVAL, "training workspace has %zu bytes, needs %zu", ws_bytes, w.total);
  hipStream_t s = (hipStream_t)hip_stream;
  char* ws = (char*)d_train_ws;
  unsigned char* blob = (unsigned char*)d_blob;
  MlpTrainOut tr;
  tr.a1 = (float*)(ws + w.a1);
  tr.a2 = (float*)(ws + w.a2);
  tr.x0t = (bf16_t*)(ws + w.x0t);
  tr.h1t = (bf16_t*)(ws + w.h1t);
  tr.h2t = (bf16_t*)(ws + w.h2t);
  tr.B = B;
  float* out = (float*)(ws + w.out);
  hipLaunchKernelGGL(k_mlp_fwd_x<true>, dim3(w.tiles), dim3(kBlock), 0, s, blob, d_X, B, out, tr);
  LAUNCH_CHECK("k_mlp_fwd_x");
  hipLaunchKernelGGL(k_mdn_grad<2>, dim3(w.groups), dim3(kBlock), 0, s, out, d_xt, B, (bf16_t*)(ws + w.gb),
                     (bf16_t*)(ws + w.gt), (float*)(ws + w.b3p), (double*)(ws + w.lossp));
  LAUNCH_CHECK("k_mdn_grad");
  MlpBwdArgs bw;
  bw.gb = (const bf16_t*)(ws + w.gb);
  bw.a1 = tr.a1;
  bw.a2 = tr.a2;
  bw.W3t = (const bf16_t*)(ws + w.w3t);
  bw.W2t = (const bf16_t*)(ws + w.w2t);
  bw.da2t = (bf16_t*)(ws + w.da2t);
  bw.da1t = (bf16_t*)(ws + w.da1t);
  bw.b2_part = (float*)(ws + w.b2p);
  bw.b1_part = (float*)(ws + w.b1p);
  bw.B = B;
  hipLaunchKernelGGL(k_mlp_bwd, dim3(w.tiles), dim3(kBlock), 0, s, bw);
  LAUNCH_CHECK("k_mlp_bwd");
  WgArgs wg;
  wg.job[0] = WgJob{bw.da1t, tr.x0t, (float*)(ws + w.wp1), kMlpHid, kMlpIn};
  wg.job[1] = WgJob{bw.da2t, tr.h1t, (float*)(ws + w.wp2), kMlpHid, kMlpHid};
  wg.job[2] = WgJob{(const bf16_t*)(ws + w.gt), tr.h2t, (float*)(ws + w.wp3), kMlpOut, kMlpHid};
  for (int j = 0; j < 3; ++j) wg.blocks[j] = (wg.job[j].M / 32) * (wg.job[j].N / 32);
  wg.B = B;
  wg.chunks = w.chunks;
  hipLaunchKernelGGL(k_mlp_wgrad, dim3(wg.blocks[0] + wg.blocks[1] + wg.blocks[2], w.chunks), dim3(kBlock), 0, s,
                     wg);
  LAUNCH_CHECK("k_mlp_wgrad");
  AdamArgs ad;
  ad.p = d_state;
  ad.m = d_state + MlpParamLayout::n;
  ad.v = d_state + 2 * MlpParamLayout::n;
  ad.grad_out = d_grad;
  ad.blob = blob;
  ad.W2t = (bf16_t*)(ws + w.w2t);
  ad.W3t = (bf16_t*)(ws + w.w3t);
  ad.wpart[0] = wg.job[0].part;
  ad.wpart[1] = wg.job[1].part;
  ad.wpart[2] = wg.job[2].part;
  ad.chunks = w.chunks;
  ad.b1_part = bw.b1_part;
  ad.b2_part = bw.b2_part;
  ad.tiles = w.tiles;
  ad.b3_part = (const float*)(ws + w.b3p);
  ad.groups = w.groups;
  ad.loss_part = (const double*)(ws + w.lossp);
  ad.loss = d_loss;
  ad.B = B;
  ad.lr = lr;
  ad.bc1 = (float)(1.0 - pow(0.9, (double)adam_t));
  ad.bc2 = (float)(1.0 - pow(0.999, (double)adam_t));
  ad.update = adam_t > 0 ? 1 : 0;
  hipLaunchKernelGGL(k_mlp_adam, dim3((MlpParamLayout::n + 255) / 256), dim3(256), 0, s, ad);
  LAUNCH_CHECK("k_mlp_adam");
  return DPF_OK;
}
