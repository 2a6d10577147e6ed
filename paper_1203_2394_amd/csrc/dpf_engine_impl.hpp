// Per-model launchers of the step kernels, instantiated by each model's
// translation unit (dpf_eng_*.hip) through DPF_DEFINE_ENGINE.
#pragma once
#include <hip/hip_runtime.h>

#include "dpf_aux.hpp"
#include "dpf_engine.hpp"
#include "dpf_kernels.hpp"
#include "dpf_learned.hpp"
#include "dpf_mlp.hpp"
#include "dpf_rb.hpp"

namespace dpf {

// Models served by the learned proposal (the network's mixture is over a
// two-dimensional x; the features must fit its input).
template <class Mdl>
constexpr bool learned_model() { return Mdl::DX == 2 && has_moments<Mdl>(); }


template <class Mdl, int SEG, int JPT>
static void launch_op(int op, const StepArgs& a, int n, hipStream_t s) {
  switch (op) {
    case OP_INIT_LA:
      hipLaunchKernelGGL((k_init<Mdl, SEG, JPT, false>), dim3(n), dim3(kBlock), 0, s, a);
      break;
    case OP_INIT_PLAIN:
      hipLaunchKernelGGL((k_init<Mdl, SEG, JPT, true>), dim3(n), dim3(kBlock), 0, s, a);
      break;
    case OP_LA_WEIGHTS:
      hipLaunchKernelGGL((k_la_weights<Mdl, SEG, JPT>), dim3(n), dim3(kBlock), 0, s, a);
      break;
    case OP_LA_WEIGHTS_NESTED:
      hipLaunchKernelGGL((k_la_weights_nested<Mdl, SEG, JPT>), dim3(n), dim3(kBlock), 0, s, a);
      break;
    case OP_DPF_WEIGHTS:
      hipLaunchKernelGGL((k_dpf_weights<Mdl, SEG, JPT>), dim3(n), dim3(kBlock), 0, s, a);
      break;
    case OP_NEWCLOUD_LA:
      hipLaunchKernelGGL((k_newcloud<Mdl, SEG, JPT, false>), dim3(n), dim3(kBlock), 0, s, a);
      break;
    case OP_NEWCLOUD_PLAIN:
      hipLaunchKernelGGL((k_newcloud<Mdl, SEG, JPT, true>), dim3(n), dim3(kBlock), 0, s, a);
      break;
    case OP_LEARNED_INNER:
      if constexpr (learned_model<Mdl>())
        hipLaunchKernelGGL((k_learned_inner<Mdl, SEG, JPT>), dim3(n), dim3(kBlock), 0, s, a);
      break;
    case OP_LA_WEIGHTS_FALLBACK:
      if constexpr (learned_model<Mdl>())
        hipLaunchKernelGGL((k_la_weights_fallback<Mdl, SEG, JPT>), dim3(n), dim3(kBlock), 0, s, a);
      break;
    case OP_NEWCLOUD_FALLBACK:
      if constexpr (learned_model<Mdl>())
        hipLaunchKernelGGL((k_newcloud_fallback<Mdl, SEG, JPT>), dim3(n), dim3(kBlock), 0, s, a);
      break;
    case OP_MOMENTS:
      if constexpr (has_moments<Mdl>())
        hipLaunchKernelGGL((k_moments<Mdl, SEG, JPT>), dim3(n), dim3(kBlock), 0, s, a, g_mom_args.y,
                           g_mom_args.feat);
      break;
  }
}

template <class Mdl>
static dpf_status engine_mlp_state(const StepArgs& a, hipStream_t s) {
  if constexpr (learned_model<Mdl>()) {
    hipLaunchKernelGGL(k_mlp_fwd_state<Mdl>, dim3((a.NT + kMlpRows - 1) / kMlpRows), dim3(kBlock), 0, s, a);
    LAUNCH_CHECK("k_mlp_fwd_state");
    return DPF_OK;
  } else {
    return fail(DPF_EUNSUPPORTED, "no learned proposal for this model");
  }
}

template <class Mdl>
static dpf_status engine_mdn_draw(const StepArgs& a, hipStream_t s) {
  if constexpr (learned_model<Mdl>()) {
    hipLaunchKernelGGL(k_mdn_draw<Mdl>, dim3((a.NT + kBlock - 1) / kBlock), dim3(kBlock), 0, s, a);
    LAUNCH_CHECK("k_mdn_draw");
    return DPF_OK;
  } else {
    return fail(DPF_EUNSUPPORTED, "no learned proposal for this model");
  }
}

template <class Mdl>
static dpf_status engine_launch(int op, const StepArgs& a, const TileClass& tc, hipStream_t s) {
  const int n = tc.n_tiles;
  switch (tc.cls) {
    case 0: launch_op<Mdl, 32, 1>(op, a, n, s); break;
    case 1: launch_op<Mdl, 64, 1>(op, a, n, s); break;
    case 2: launch_op<Mdl, 128, 1>(op, a, n, s); break;
    case 3: launch_op<Mdl, 64, 4>(op, a, n, s); break;
    case 4: launch_op<Mdl, 256, 4>(op, a, n, s); break;
    case 5: launch_op<Mdl, 256, 16>(op, a, n, s); break;
    case 6: launch_op<Mdl, 32, 2>(op, a, n, s); break;
    case 7: launch_op<Mdl, 32, 4>(op, a, n, s); break;
    case 8: launch_op<Mdl, 64, 2>(op, a, n, s); break;
    case 9: launch_op<Mdl, 256, 1>(op, a, n, s); break;
    case 10: launch_op<Mdl, 128, 2>(op, a, n, s); break;
    case 11: launch_op<Mdl, 16, 2>(op, a, n, s); break;
    case 12: launch_op<Mdl, 16, 4>(op, a, n, s); break;
    case 13: launch_op<Mdl, 16, 8>(op, a, n, s); break;
    default: return fail(DPF_EUNSUPPORTED, "no kernel class %d", tc.cls);
  }
  LAUNCH_CHECK("step kernel");
  return DPF_OK;
}

template <class Mdl>
static dpf_status engine_rb(const StepArgs& a, double* tmp, float* out, hipStream_t s) {
  constexpr int per = kBlock / kWave;  // outer particles per workgroup
  hipLaunchKernelGGL(k_rb_outer<Mdl>, dim3((a.NT + per - 1) / per), dim3(kBlock), 0, s, a, tmp);
  LAUNCH_CHECK("k_rb_outer");
  hipLaunchKernelGGL(k_rb_finish<Mdl::DX>, dim3(a.n_filters), dim3(kBlock), 0, s, a, (const double*)tmp, out);
  LAUNCH_CHECK("k_rb_finish");
  return DPF_OK;
}

template <class Mdl>
static dpf_status engine_finalize(const StepArgs& a, int F, hipStream_t s) {
  constexpr int DX = Mdl::DX, DZ = Mdl::DZ;
  hipLaunchKernelGGL((k_finalize<DX, DZ, true>), dim3(F), dim3(fin_block<DX, DZ>()), 0, s, a);
  LAUNCH_CHECK("k_finalize");
  return DPF_OK;
}

template <class Mdl, bool YH>
static dpf_status engine_post_y(const StepArgs& a, const int2* rg, int n_rgroups, int F, int next, int split,
                                hipStream_t s) {
  constexpr int DX = Mdl::DX, DZ = Mdl::DZ;
  hipLaunchKernelGGL((k_post<DX, DZ, YH>), dim3(n_rgroups), dim3(kBlock), 0, s, a, rg, next, split);
  LAUNCH_CHECK("k_post");
  if (split) {
    hipLaunchKernelGGL((k_post_end<DX, DZ, YH>), dim3(F), dim3(kWave), 0, s, a, next);
    LAUNCH_CHECK("k_post_end");
  }
  return DPF_OK;
}

// (the predicted observation's partial sums when the step formed them)
template <class Mdl>
static dpf_status engine_post(const StepArgs& a, const int2* rg, int n_rgroups, int F, int next, int split,
                              hipStream_t s) {
  if constexpr (has_yhat<Mdl>()) {
    if (a.yp != nullptr) return engine_post_y<Mdl, true>(a, rg, n_rgroups, F, next, split, s);
  }
  return engine_post_y<Mdl, false>(a, rg, n_rgroups, F, next, split, s);
}

// The engine table entry of model Mdl with parameter derivation DERIVE.
template <class Mdl>
static Engine make_engine(void (*derive)(const double*, std::vector<float>&)) {
  return Engine{Mdl::DX,
                Mdl::DZ,
                Mdl::DY,
                (size_t)Mdl::L::n_raw,
                (size_t)Mdl::L::n_total,
                derive,
                engine_launch<Mdl>,
                learned_model<Mdl>() ? engine_mlp_state<Mdl> : nullptr,
                learned_model<Mdl>() ? engine_mdn_draw<Mdl> : nullptr,
                has_moments<Mdl>(),
                engine_rb<Mdl>,
                engine_finalize<Mdl>,
                engine_post<Mdl>,
                has_yhat<Mdl>()};
}

}  // namespace dpf
