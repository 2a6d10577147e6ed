/*
 * dpf.h -- C interface of the MI355X (gfx950) look-ahead decentralized
 * particle filter library (libdpf.so).
 *
 * Method: Ahmed, Bibalan, de Freitas, Fauvel, "Decentralized, Adaptive,
 * Look-Ahead Particle Filtering", arXiv:1203.2394.
 *
 * Problem statement (Section 2, Eq. (1)): a state split into an outer block
 * x (dimension dx) and an inner block z (dz) with observations y (dy),
 *     x_{t+1} = f^x(x_t, z_t, v^x),  z_{t+1} = f^z(x_{t:t+1}, z_t, v^z),
 *     y_t = h(x_t, z_t, e_t),
 * with known parameters.  Following the factorisation Eq. (2), a filter
 * keeps N outer particles x^{(i)}, each carrying a conditional particle
 * filter of M inner particles z^{(i,j)} with normalised log-weights
 * log qbar^{(i,j)} (eq:qbar).  One call advances every filter of a handle by
 * one time step.
 *
 * Conventions for every function below:
 *  - "d_" pointers are device memory of the GPU current when the handle was
 *    created; "h_" or unprefixed pointers in dpf_config are host memory.
 *  - The caller owns all device memory (workspace, inputs, outputs); the
 *    library never allocates device memory (its one device array, the 8 KiB
 *    of dpf_systematic_noalloc, is part of the loaded code object).  Buffers
 *    must stay valid until the work queued on the handle's stream has
 *    finished.
 *  - All calls are asynchronous on the handle's HIP stream and return after
 *    queueing.  Argument and launch errors return synchronously with a
 *    non-zero dpf_status and a message from dpf_last_error(); conditions
 *    that depend on the data never fail a call -- they set per-filter flag
 *    bits (DPF_FLAG_*), readable with dpf_estimate.
 *  - A handle is not thread-safe; distinct handles are independent.
 *  - Floating point: particle state in FP32; normalisations, scans,
 *    evidence and estimates accumulated in FP64.
 *  - Random numbers: Philox4x32-10 keyed by (seed, filter index) with
 *    counters (t, outer index, inner index, purpose); results are a pure
 *    function of (config, observations) and reproducible bit for bit.
 */
#ifndef DPF_H
#define DPF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DPF_ABI_VERSION 1u

typedef struct dpf_handle dpf_handle; /* opaque; host memory; freed by dpf_destroy */

typedef enum {
  DPF_OK = 0,
  DPF_EINVAL = 1,       /* bad argument (null pointer, size, mismatch)        */
  DPF_ENOMEM = 2,       /* workspace too small                                */
  DPF_EDEVICE = 3,      /* a HIP call failed (message names it)               */
  DPF_ESTATE = 4,       /* call not valid for this handle (e.g. wrong algo)   */
  DPF_EUNSUPPORTED = 5  /* model / dimensions / sizes not built into library  */
} dpf_status;

/* Models (parameter blob layouts; all values double, copied at create):
 *
 * DPF_MODEL_LINGAUSS -- linear-Gaussian, built for (dx,dz,dy) = (1,2,1):
 *   Ax[dx*dx] Cxz[dx*dz] qx Az[dz*dz] Bzx[dz*dx] qz Hx[dy*dx] Hz[dy*dz] r
 *   x' = Ax x + Cxz z + sqrt(qx) v ; z' = Az z + Bzx x' + sqrt(qz) w ;
 *   y = Hx x + Hz z + sqrt(r) e.                      (row-major matrices)
 * DPF_MODEL_NONLIN -- built for (dx,dz,dy) = (2,8,8):
 *   a b qx W[dz*dx] rho qz c r bmode
 *   x'_d = a x_d + b x_d/(1+x_d^2) + sqrt(qx) v_d ;
 *   z' = tanh(W x') + rho z + sqrt(qz) w ;
 *   y_k = z_k + c g_k(x) + sqrt(r) e_k, g_k = x_{k mod dx}^2 (bmode 0) or
 *   |x|^2 (bmode 1).
 * DPF_MODEL_HIGHDIM -- built for (dx,dz,dy) = (4,64,32):
 *   a b qx Alo[dz-1] Adiag[dz] Aup[dz-1] B[dz*dx] qz C[dy*dz] r eps nu gonly
 *   x' as NONLIN ; z' = A z + B sin(x') + sqrt(qz) w, A tridiagonal ;
 *   y = C z + e, each e_k with density (1-eps) N(0,r) + eps t_nu(e/sqrt r)/sqrt r
 *   (gonly != 0: plain N(0, r)).
 * DPF_MODEL_TWODIM -- model 1 of Table 1 (the 2-dimensional example), built
 *   for (dx,dz,dy) = (1,1,1):
 *   qx qz cxz rho b amp freq r tswap
 *   x' = x + z/(1+z^2) + v^x ;
 *   z' = x + rho z + b z/(1+z^2) + amp cos(freq t) + v^z, t the time of the
 *   state the transition leaves ;
 *   (v^x, v^z) ~ N(0, [[qx, cxz], [cxz, qz]]) ; y = atan(x) + z^2/20 + e,
 *   e ~ N(0, r).  Table 1's values: 1 1 0.1 0.5 25 8 1.2 1.  From t >= tswap
 *   on the two transition laws are swapped (the change point of Section
 *   4.3): x' = z + rho x + b x/(1+x^2) + amp cos(freq t) + v^x,
 *   z' = z + x/(1+x^2) + v^z (tswap = +inf: never).  Needs qx, qz, r > 0
 *   and qx qz > cxz^2 (else DPF_EINVAL).  x is sampled first (outer).
 * DPF_MODEL_TWODIM_ZFIRST -- the same model and parameter blob, z sampled
 *   first (the other decomposition of Section 3 / 4.3): the outer state is
 *   z, the inner state x, so xmean estimates z and zmean estimates x.
 * DPF_MODEL_FOURDIM -- model 2 of Table 1 (the 4-dimensional example), built
 *   for (dx,dz,dy) = (2,2,1):
 *   a1 bs c21 a2 qx1 qx2 qz1 qz2 cz rho b amp freq r
 *   x1' = a1 x1 + bs sin t + v1 ; x2' = c21 x1 + a2 x2 + v2 ;
 *   z1' = z1 + z2/(1+z2^2) + w1 ; z2' = z1' + rho z2 + b z2/(1+z2^2) +
 *   amp cos(freq t) + w2, t the time of the state the transition leaves ;
 *   v ~ N(0, diag(qx1, qx2)), (w1, w2) ~ N(0, [[qz1, cz], [cz, qz2]]) ;
 *   y = (x1 + x2)/(1 + x1^2) + atan(z1) + z2^2/20 + e, e ~ N(0, r).
 *   Table 1's values: 0.5 8 0.4 0.5 1 1 1 10 0.1 0.5 25 8 1.2 1.  Needs
 *   positive variances and qz1 qz2 > cz^2 (else DPF_EINVAL).
 * Every model has the prior [x_0; z_0] ~ N(0, I).
 */
typedef enum {
  DPF_MODEL_LINGAUSS = 1,
  DPF_MODEL_NONLIN = 2,
  DPF_MODEL_HIGHDIM = 3,
  DPF_MODEL_TWODIM = 4,
  DPF_MODEL_FOURDIM = 5,
  DPF_MODEL_TWODIM_ZFIRST = 6
} dpf_model;

/* Which filter a handle runs. */
typedef enum {
  DPF_ALGO_LOOKAHEAD = 0, /* look-ahead DPF (Fig. 4); also the learned step */
  DPF_ALGO_PLAIN = 1      /* DPF with prior proposals (Fig. 2)              */
} dpf_algo;

/* Per-filter flag bits (latched until dpf_reset / dpf_create). */
#define DPF_FLAG_DEGENERATE_OUTER 1u /* no finite outer weight: uniform resampling used */
#define DPF_FLAG_DEGENERATE_INNER 2u /* an inner cloud had no finite weight: uniform    */
#define DPF_FLAG_NONFINITE 4u        /* NaN / +inf weight or non-finite observation     */
#define DPF_FLAG_FALLBACK 8u         /* learned step fell back to the look-ahead step   */

typedef struct {
  uint32_t abi_version;  /* DPF_ABI_VERSION                                  */
  int32_t model;         /* dpf_model                                        */
  int32_t algo;          /* dpf_algo                                         */
  int32_t dx, dz, dy;    /* must match a built (model, dims) combination     */
  const double* params;  /* host, n_params values in the model's blob layout */
  size_t n_params;
  int32_t n_filters;     /* F >= 1 independent filters                       */
  const int32_t* N;      /* host [F]: outer particles per filter, 1..65536   */
  const int32_t* M;      /* host [F]: inner particles per filter, 1..4096    */
  uint64_t seed;         /* Philox key; filter f uses key (seed, f)          */
  uint32_t reserved;     /* must be 0                                        */
} dpf_config;

/* Bytes of device workspace a handle with this config needs (0 on error). */
size_t dpf_workspace_bytes(const dpf_config* cfg);

/* Validate cfg, carve d_workspace (>= dpf_workspace_bytes, 256-byte
 * aligned), upload parameters and queue the initialisation (prior draws at
 * t = 0, Fig. 2 / Fig. 4 "Initialize"; the plain DPF also proposes t = 1
 * from the prior since no y_0 is observed).  hip_stream: hipStream_t or
 * NULL for the default stream.  On success *out owns host state only. */
dpf_status dpf_create(const dpf_config* cfg, void* d_workspace, size_t bytes, void* hip_stream,
                      dpf_handle** out);

/* Queue the initialisation again (t = 0, flags and evidence cleared). */
dpf_status dpf_reset(dpf_handle* h);

/* Release host state (does not synchronise or free the workspace). */
dpf_status dpf_destroy(dpf_handle* h);

/* One look-ahead DPF step (Section 2.2, Fig. 4, steps 1-4) for every active
 * filter, consuming y_t for its next t: look-ahead weights eq:weightsMC over
 * each outer particle's inner cloud, systematic outer resampling at t-1,
 * new x from the Monte Carlo optimal proposal eq:approx3 (SIR over the
 * look-ahead candidates), x-conditioned local inner resampling eq:qnobar,
 * inner propagation and the inner measurement update eq:qbar.
 * d_y: [F][dy] float.  d_active: [F] bytes (0 = skip this filter) or NULL.
 * Requires algo DPF_ALGO_LOOKAHEAD. */
dpf_status dpf_lookahead_step(dpf_handle* h, const float* d_y, const uint8_t* d_active);

/* One plain DPF step (Section 2, Fig. 2, steps 1-7, prior proposals of
 * Section 2.1) consuming y_t: weights (eq:approx2), estimates, systematic
 * outer resampling, x proposal from eq:approx1, eq:qnobar inner
 * resampling and inner proposal.  Same arguments as dpf_lookahead_step.
 * Requires algo DPF_ALGO_PLAIN. */
dpf_status dpf_step(dpf_handle* h, const float* d_y, const uint8_t* d_active);

/* Copy the estimates of each filter's last step (any pointer may be NULL):
 * d_xmean [F][dx], d_zmean [F][dz] float (posterior means), d_ess [F] float
 * (effective sample size of the outer weights used for resampling),
 * d_loglik [F] double (cumulative log evidence, sum over steps of
 * logsumexp_i log w_i - log N), d_flags [F] uint32 (DPF_FLAG_* bits). */
dpf_status dpf_estimate(dpf_handle* h, float* d_xmean, float* d_zmean, float* d_ess,
                        double* d_loglik, uint32_t* d_flags);

/* Run up to T steps of the handle's algorithm over device-resident
 * observations, each filter f stepping while its time is below
 * min(T_f, T).  d_Y: [T][F][dy] float, row t-1 holding y_t of every filter
 * (absolute time).  d_Tf: [F] int32 or NULL (all T).  d_xtrace [T][F][dx]
 * and d_ztrace [T][F][dz] (or NULL) receive the per-step estimates at row
 * t-1.  use_graph != 0 runs the first step directly, then captures a chunk
 * of min(T - 1, 256) steps into a HIP graph once and replays it (the step's
 * launches read every per-filter time and buffer choice from device memory,
 * so replays need no host work), and the steps the chunks do not cover as a
 * second captured graph; both are cached for the next run of the same
 * length and buffers.
 * A look-ahead run takes Fig. 4 steps 1-2 of step t+1 (the look-ahead
 * weights, eq:weightsMC) inside step t's new-cloud launch, from the clouds
 * it has just built, and the outer-weight statistics of step t+1 inside step
 * t's step-end launch: results are bit-identical to T dpf_lookahead_step
 * calls with the same activity (per-filter horizons included). */
dpf_status dpf_run(dpf_handle* h, const float* d_Y, int32_t T, const int32_t* d_Tf,
                   float* d_xtrace, float* d_ztrace, int32_t use_graph);

/* Nested look-ahead estimator (Section 2.1 after eq:approx3; Fig. 4 step 1
 * with N_z' > 1 companions per candidate, eq:weightsMC).  n_comp = K >= 1:
 * the look-ahead weight of every candidate x^{(i,m)} (drawn from inner
 * component m, LA_X at (t, i, m)) averages p(y_t | x^{(i,m)}, z) over K
 * companions z drawn from the inner predictive given the candidate -- their
 * ancestors by systematic resampling (U53 of purpose LA_B = 13 at (t, i, m))
 * of the inner weights conditioned on the candidate as in eq:qnobar, their
 * propagation with LA_Z normals k dz .. k dz + dz - 1 at (t, i, m) (block-
 * aligned layout: normal n from Philox block n / 4):
 *   ell^{(i,m)} = log qbar^{(i,m)} + log (1/K) sum_k p(y_t | x^{(i,m)}, z^{(i,m,k)}).
 * n_comp = 0 (the default): one companion drawn together with the candidate
 * from the same inner component (normals dx .. dx + dz - 1 of the candidate's
 * LA_X draw).  1 <= K <= 1024; DPF_ESTATE for a plain
 * handle.  Takes effect from the next dpf_lookahead_step / dpf_run (a run
 * with K >= 1 takes each step whole instead of computing the next step's
 * weights inside the new-cloud launch; results still equal step calls).  Cost
 * per outer particle: K M model evaluations, K M^2 where p(x' | x, z) depends
 * on z.  The learned step's fallback keeps the paired form. */
dpf_status dpf_set_lookahead_companions(dpf_handle* h, int32_t n_comp);

/* Predicted observation (the one-step-ahead prediction whose error is the
 * reward of the decomposition choice, Section 3 and Section 4.3):
 *   yhat_{t|t-1} = (1/N) sum_i sum_j qbar^{(i,j)} h(x^{(i,j)}, z^{(i,j)}),
 * the look-ahead draws of Fig. 4 step 1 weighted as draws from the one-step
 * predictive p(x_t, z_t | y_{0:t-1}) (nested estimator: h averaged over each
 * candidate's companions); h the noise-free observation.  enable != 0: every
 * following look-ahead step (dpf_lookahead_step, dpf_run) forms it from
 * its own look-ahead draws; d_ytrace [T][F] float (or NULL) receives it at
 * row t-1 as y_t is consumed.  Built for models with a one-dimensional y
 * (LINGAUSS, TWODIM, TWODIM_ZFIRST, FOURDIM; else DPF_EUNSUPPORTED); look-ahead
 * handles only (DPF_ESTATE); not formed by the learned step. */
dpf_status dpf_set_prediction(dpf_handle* h, int32_t enable, float* d_ytrace);

/* Copy the predicted observation of each filter's last look-ahead step:
 * d_yhat [F] float (DPF_ESTATE unless dpf_set_prediction enabled it). */
dpf_status dpf_predicted_observation(dpf_handle* h, float* d_yhat);

/* Rao-Blackwellised estimate of the new outer state of the look-ahead step
 * just taken: xhat_rb = sum_i Wbar_i sum_j pi_ij xla^{(i,j)}, Wbar the
 * normalised look-ahead weights (eq:weightsMC), pi_i. = softmax_j ell_ij the
 * candidate probabilities of eq:approx3's sampling-importance-resampling,
 * xla the look-ahead candidates (regenerated from their random streams) --
 * the expectation of the particle that outer resampling and the candidate
 * draw produce, without their sampling noise.  d_xrb: device float
 * [F][dx], written on the handle's stream; NaN for filters that sat the
 * step out.  Valid only directly after dpf_lookahead_step (DPF_ESTATE after
 * any other state change: a run, a learned step, an import, a reset). */
dpf_status dpf_estimate_rb(dpf_handle* h, float* d_xrb);

/* State import / export (checkpoint, and step-level comparisons).  Layout,
 * all little-endian: int32 t[F] padded to a multiple of 16 bytes, then
 * float x[dx][sum N], float z[sum_f N_f*dz*M_f] (filter blocks in order,
 * each [N][dz][M]), float lam[sum_f N_f*M_f] (log qbar, [N][M] per filter).
 * For DPF_ALGO_PLAIN, x and z are the proposals for the next step and lam
 * is unused.  Import resets the flags and the cumulative evidence. */
size_t dpf_state_bytes(const dpf_handle* h);
dpf_status dpf_export_state(dpf_handle* h, void* d_dst, size_t bytes);
dpf_status dpf_import_state(dpf_handle* h, const void* d_src, size_t bytes);

/* Internal buffers of the last step, copied out for inspection:
 * DPF_BUF_ELL  float [sum N*M]: look-ahead (or measurement) log-weights ell
 *                               of the last step taken (also after a run)
 * DPF_BUF_LOGW float [sum N]:   outer log-weights log w_i of that step
 * DPF_BUF_ANC  int32 [sum N]:   outer ancestors A_k
 * DPF_BUF_SEL  int32 [sum N]:   selected candidate (look-ahead) or
 *                               inner ancestor a_k (plain) per new particle;
 *                               after a learned step, the mixture component
 *                               drawn for each pre-resampling particle
 * DPF_BUF_MDN  float [sum N][32]: network outputs of the last learned step
 * DPF_BUF_X    float [dx][sum N]: outer particles x of the current state
 * DPF_BUF_FALLBACK uint8 [F]:   1 where the last learned step fell back to
 *                               the look-ahead step (0 for filters that were
 *                               inactive or kept the learned proposals) */
typedef enum {
  DPF_BUF_ELL = 0,
  DPF_BUF_LOGW = 1,
  DPF_BUF_ANC = 2,
  DPF_BUF_SEL = 3,
  DPF_BUF_MDN = 4,
  DPF_BUF_X = 5,
  DPF_BUF_FALLBACK = 6
} dpf_buffer;
dpf_status dpf_copy_buffer(dpf_handle* h, int32_t which, void* d_dst, size_t bytes);

/* Phase timing.  hip_events: n_events hipEvent_t handles created by the
 * caller (n_events a multiple of 5), or NULL / 0 to stop.  Each following
 * step call (dpf_step, dpf_lookahead_step, and every step of dpf_run without
 * a graph) records the next 5 events on the handle's stream: before the
 * weight kernels, after them, after the outer resampling, after the
 * new-cloud kernels and after the estimates, until the array is used up.
 * Elapsed times between consecutive events give each phase's duration. */
dpf_status dpf_set_phase_events(dpf_handle* h, void* const* hip_events, int32_t n_events);

/* Message for the last non-OK status returned on this thread. */
const char* dpf_last_error(void);

/* ---- tiling ----
 * Per-particle kernels run 256-thread workgroups split into segments of SEG
 * lanes, one outer particle per segment, each lane handling JPT inner
 * particles (a class holds M <= SEG * JPT).  dpf_tile_classes writes the
 * built classes' (SEG, JPT) into seg / jpt (up to n entries, either may be
 * NULL) and returns their number.  By default a filter uses the first of
 * classes 0..5 that holds its M. */
int32_t dpf_tile_classes(int32_t* seg, int32_t* jpt, int32_t n);

/* Choose the class of each filter: h_cls [F] host, a class index holding the
 * filter's M, or -1 for the default.  Takes effect for the following calls
 * (results then depend on the class only through floating-point reduction
 * order); a captured run graph is rebuilt. */
dpf_status dpf_set_tiling(dpf_handle* h, const int32_t* h_cls);

/* ---- learned proposal for the outer block ----
 *
 * A mixture density network q(x_t | features) stands in for the Monte Carlo
 * optimal-proposal estimate eq:approx3.  Features of outer particle i (raw,
 * standardised with the mean / standard deviation stored in the blob):
 *   [x_{t-1}^{(i)} (dx), y_t (dy), sum_j qbar z^{(i,j)} (dz),
 *    sum_j qbar (z^{(i,j)} - mean)^2 (dz)], zero-padded to 32.
 * Network 32 -> 256 -> 256 -> 32 with tanh-form GELU after the hidden
 * layers, BF16 matrix-core arithmetic with FP32 accumulation.  Outputs (20
 * of 32 used, dx = 2): 4 mixture logits, 4 x 2 means, 4 x 2 log standard
 * deviations (clamped to [log 1e-3, log 1e3]), component-major.
 * Built for DPF_MODEL_NONLIN.
 *
 * Blob (device, DPF_MLP_BLOB_BYTES, byte offsets): W1 bf16 [256][32] at 0,
 * W2 bf16 [256][256] at 16384, W3 bf16 [32][256] at 147456, b1 float [256]
 * at 163840, b2 float [256] at 164864, b3 float [32] at 165888, feature
 * mean float [32] at 166016, feature standard deviation float [32] at
 * 166144 (BF16: round to nearest even of the FP32 value).
 * Parameter vector (FP32, DPF_MLP_NPARAM values, training): W1 [256][32],
 * b1 [256], W2 [256][256], b2 [256], W3 [32][256], b3 [32]. */
#define DPF_MLP_BLOB_BYTES 166272u
#define DPF_MLP_NPARAM 82464u

/* Copy the network blob into the handle (the caller may free d_blob once
 * the stream has passed this call) and set the fallback threshold: a
 * filter whose learned outer weights have ESS < ess_frac * N (or no finite
 * weight) takes the look-ahead step instead (ess_frac in [0, 1]).  Queues
 * the cloud moments of the current state.  Look-ahead handles only. */
dpf_status dpf_set_proposal(dpf_handle* h, const void* d_blob, size_t bytes, double ess_frac);

/* One step with the learned proposal (importance-sampling step of Fig. 2,
 * step 1, with q in place of the prior) for every active filter: x_t ~ q
 * (component: U53 of purpose MDN_U at (t, i); normals MDN_X at (t, i, 0)),
 * inner cloud conditioned on x_t (eq:qnobar) and resampled (INNER_U at
 * (t, i)), propagated (NEW_Z at (t, i, j)) and updated (eq:qbar), outer
 * log-weight log p_Nz(y_t | .) (eq:approx2) + log p_Nz(x_t | .)
 * (eq:approx1) - log q(x_t), systematic outer resampling (OUTER_U).
 * Filters below the ESS threshold run dpf_lookahead_step's step from the
 * unchanged state and get DPF_FLAG_FALLBACK.  Same arguments as
 * dpf_lookahead_step; needs dpf_set_proposal first. */
dpf_status dpf_learned_step(dpf_handle* h, const float* d_y, const uint8_t* d_active);

/* As dpf_learned_step with the network outputs supplied by the caller:
 * d_mdn [sum N][32] float (row i: the mixture for pre-resampling particle
 * i), and the threshold ess_frac for this call.  For checks of the step
 * against a reference and for callers with their own proposal. */
dpf_status dpf_learned_step_given(dpf_handle* h, const float* d_y, const uint8_t* d_active,
                                  const float* d_mdn, double ess_frac);

/* dpf_run with the learned step: up to T learned steps over device-resident
 * observations d_Y [T][F][dy] (same arguments and graph replay as dpf_run);
 * needs dpf_set_proposal first. */
dpf_status dpf_learned_run(dpf_handle* h, const float* d_Y, int32_t T, const int32_t* d_Tf,
                           float* d_xtrace, float* d_ztrace, int32_t use_graph);

/* Raw (unstandardised) features of every outer particle of the current
 * state for observations d_y [F][dy]: d_feat [sum N][32] float, zero-padded
 * (cloud moments by an exact two-pass reduction). */
dpf_status dpf_features(dpf_handle* h, const float* d_y, float* d_feat);

/* Sizes of the blob and of the parameter vector. */
size_t dpf_mlp_blob_bytes(void);
size_t dpf_mlp_param_count(void);

/* Network outputs for B rows of standardised features: d_X [B][32] float
 * (rounded to BF16 on load) -> d_out [B][32] float. */
dpf_status dpf_mlp_forward(const void* d_blob, const float* d_X, int32_t B, float* d_out, void* hip_stream);

/* Device workspace of one training step with batch B (a multiple of 32, at
 * most 2^20); 0 for an invalid B. */
size_t dpf_mlp_train_workspace_bytes(int32_t batch);

/* Write the blob from FP32 parameters d_params [DPF_MLP_NPARAM] and the
 * feature standardisation d_fmean, d_fstd [32] (pad entries: mean 0,
 * standard deviation 1).  d_train_ws (or NULL): a training workspace, whose
 * transposed weight copies are initialised too -- required before the
 * first dpf_mlp_train_step with that workspace. */
dpf_status dpf_mlp_pack(const float* d_params, const float* d_fmean, const float* d_fstd, void* d_blob,
                        void* d_train_ws, size_t ws_bytes, void* hip_stream);

/* One training step on a batch: mean negative log-likelihood of the
 * mixture at the targets d_xt [B][2] for standardised features d_X [B][32],
 * its gradient (forward and backward on the matrix cores, BF16 operands,
 * FP32 accumulation), then Adam (beta 0.9, 0.999, eps 1e-8, learning rate
 * lr, bias corrections for step adam_t >= 1) on the FP32 state
 * d_state [3][DPF_MLP_NPARAM] (parameters, first and second moments), and
 * the updated blob d_blob.  adam_t = 0 computes the loss and gradient
 * only.  d_loss [1] (mean NLL before the update) and d_grad
 * [DPF_MLP_NPARAM] may be NULL.  d_train_ws: dpf_mlp_train_workspace_bytes
 * bytes, initialised by dpf_mlp_pack. */
dpf_status dpf_mlp_train_step(float* d_state, void* d_blob, const float* d_X, const float* d_xt, int32_t B,
                              float lr, int32_t adam_t, void* d_train_ws, size_t ws_bytes, float* d_loss,
                              float* d_grad, void* hip_stream);

/* ---- the training set of the learned proposal (pairs the look-ahead DPF
 * generates; training-loop plumbing, not the filter's arithmetic) ---- */

/* Mean and sample standard deviation (divisor n - 1, floored at std_floor
 * >= 0) of each of the first `cols` columns of d_X [n][ld] float, row-major:
 * d_mean, d_std [cols].  FP64 sums in a fixed order (the same bits on every
 * call).  n >= 2, 1 <= cols <= ld. */
dpf_status dpf_feature_stats(const float* d_X, int64_t n, int32_t cols, int32_t ld, float* d_mean,
                             float* d_std, float std_floor, void* hip_stream);

/* d_out [n][ld_out] = (X - mean) / std in the first `cols` columns (FP32,
 * IEEE division), 0 in the others (the network's zero-padded inputs). */
dpf_status dpf_standardize(const float* d_X, int64_t n, int32_t cols, int32_t ld, const float* d_mean,
                           const float* d_std, float* d_out, int32_t ld_out, void* hip_stream);

/* d_perm [n] int32: a pseudo-random permutation of 0..n-1 keyed by (seed,
 * epoch) -- a four-round Feistel network on the smallest even number of
 * bits that covers n, walked until the value falls below n.  The same
 * (seed, epoch, n) always gives the same permutation.  0 <= n < 2^31. */
dpf_status dpf_permutation(uint64_t seed, uint32_t epoch, int64_t n, int32_t* d_perm, void* hip_stream);

/* d_dst [count][ld_dst] = rows d_idx[0..count) of d_src [n_src][ld_src]
 * (first `cols` columns).  An index outside 0..n_src-1 gives a row of NaN
 * (no read outside d_src). */
dpf_status dpf_gather_rows(const float* d_src, int64_t n_src, int32_t cols, int32_t ld_src,
                           const int32_t* d_idx, int32_t count, float* d_dst, int32_t ld_dst,
                           void* hip_stream);

/* ---- kernel-level primitives (same device code as the step kernels) ---- */

/* Philox4x32-10 words: d_ctr [n][4] uint32 counters -> d_out [n][4] words
 * under key (seed_lo32, seed_hi32 ^ filter_id). */
dpf_status dpf_philox_words(uint64_t seed, uint32_t filter_id, const uint32_t* d_ctr, size_t n,
                            uint32_t* d_out, void* hip_stream);

/* FP32 standard normals of the random-number contract: d_out [n_a][n_b][D]
 * = normal d of counter (t, a, b, purpose) for a < n_a, b < n_b, in the
 * packed layout (ten normals per two Philox blocks: normals 10q .. 10q+7
 * from the words of blocks 2q and 2q+1, normals 10q+8 and 10q+9 from the two
 * blocks' remnant uniforms).  D in {1, 2, 4, 8, 10, 64, 68}, else
 * DPF_EUNSUPPORTED. */
dpf_status dpf_normals(uint64_t seed, uint32_t filter_id, uint32_t t, uint32_t purpose, int32_t n_a,
                       int32_t n_b, int32_t D, float* d_out, void* hip_stream);

/* Systematic resampling of one weight vector by the outer-resampling code:
 * d_w [n] non-negative doubles (not all zero), n <= 65536, points
 * ((k + u) C) / n_out, d_out[k] = first i with C_i > point (C = inclusive
 * FP64 cumulative sum; a point at or past the total takes the first i with
 * C_i reaching it).  d_scratch: 4 * ceil(n / 256) doubles of device memory
 * (per-group statistics). */
dpf_status dpf_systematic(const double* d_w, int32_t n, int32_t n_out, double u, double* d_scratch,
                          int32_t* d_out, void* hip_stream);

/* dpf_systematic without a scratch argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, rule and results as
 * dpf_systematic; the group statistics live in a library-owned device array
 * of 4 * 256 doubles (8 KiB) per GPU, held until the process ends, so n is at
 * most 65536 (larger n: DPF_EUNSUPPORTED).  Allocates nothing.  Every call
 * on a GPU uses that GPU's one array: calls that may overlap on one GPU
 * (different streams, host threads) race and must be serialised by the
 * caller; calls queued on one stream are ordered. */
dpf_status dpf_systematic_noalloc(const double* d_w, int32_t n, int32_t n_out, double u, int32_t* d_out,
                                  void* hip_stream);

/* The same rule per segment by the inner-resampling code: d_w [S][n]
 * doubles, d_u [S], n_out = n (local resampling) or 1 (single draw);
 * d_out [S][n_out].  n <= 4096. */
dpf_status dpf_segmented_systematic(const double* d_w, int32_t S, int32_t n, int32_t n_out,
                                    const double* d_u, int32_t* d_out, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* DPF_H */
