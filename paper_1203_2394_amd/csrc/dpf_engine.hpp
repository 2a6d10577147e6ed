// Host-side interface between the library's C entry points (dpf_lib.hip) and
// the per-model translation units (dpf_eng_*.hip), each of which instantiates
// the step kernels of one model for every tile class and exposes them through
// an Engine table.  Splitting the models over translation units lets them
// compile in parallel.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/dpf.h"
#include "dpf_kernels.hpp"

namespace dpf {

// Record a failure message for dpf_last_error and return s.
dpf_status fail(dpf_status s, const char* fmt, ...);

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(DPF_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define LAUNCH_CHECK(what)                                                                 \
  do {                                                                                     \
    hipError_t e_ = hipGetLastError();                                                     \
    if (e_ != hipSuccess) return fail(DPF_EDEVICE, "launch of %s failed: %s", what, hipGetErrorString(e_)); \
  } while (0)

// ------------------------------------------------------------ tile classes
struct ClassShape {
  int seg, jpt;
};
// The first six are the defaults (the first that holds M); the others are
// chosen only by dpf_set_tiling (an autotuner).  For 129..256 inner particles
// the default is one wave per outer particle with four inner particles per
// lane, which measured faster than a 256-lane workgroup per particle.
static constexpr ClassShape kClasses[] = {{32, 1}, {64, 1}, {128, 1}, {64, 4},  {256, 4}, {256, 16},
                                          {32, 2}, {32, 4}, {64, 2},  {256, 1}, {128, 2},
                                          {16, 2}, {16, 4}, {16, 8}};
constexpr int kNumClasses = 14;
constexpr int kNumDefaultClasses = 6;

struct TileClass {
  int cls;
  int n_tiles;
  int4* d_tiles;
};

enum Op {
  OP_INIT_LA,
  OP_INIT_PLAIN,
  OP_LA_WEIGHTS,
  OP_DPF_WEIGHTS,
  OP_NEWCLOUD_LA,
  OP_NEWCLOUD_PLAIN,
  OP_LEARNED_INNER,
  OP_MOMENTS,
  OP_LA_WEIGHTS_FALLBACK,
  OP_NEWCLOUD_FALLBACK,
  OP_LA_WEIGHTS_NESTED
};

// Extra arguments of OP_MOMENTS (feature rows for dpf_features).
struct MomArgs {
  const float* y;
  float* feat;
};
extern thread_local MomArgs g_mom_args;

// ------------------------------------------------------------ model engines
struct Engine {
  int dx, dz, dy;
  size_t n_raw;
  size_t n_total;
  void (*derive)(const double* raw, std::vector<float>& out);
  dpf_status (*launch)(int op, const StepArgs& a, const TileClass& tc, hipStream_t s);
  dpf_status (*mlp_state)(const StepArgs& a, hipStream_t s);  // null: no learned proposal
  dpf_status (*mdn_draw)(const StepArgs& a, hipStream_t s);
  bool moments;
  dpf_status (*rb)(const StepArgs& a, double* tmp, float* out, hipStream_t s);
  // plain DPF estimates (one workgroup per filter)
  dpf_status (*finalize)(const StepArgs& a, int F, hipStream_t s);
  // look-ahead step end over n_rgroups resampling groups; split: group pass
  // and a per-filter pass as two launches
  dpf_status (*post)(const StepArgs& a, const int2* rgroups, int n_rgroups, int F, int next, int split,
                     hipStream_t s);
  bool yhat;  // the look-ahead pass can form the predicted observation
};

extern const Engine kEngLinGauss, kEngNonLin, kEngHighDim, kEngTwoDim, kEngFourDim, kEngTwoDimZ;

}  // namespace dpf
