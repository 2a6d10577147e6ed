#!/usr/bin/env python3
"""Throughput benchmark of the look-ahead DPF step on one MI355X, with the
learned-proposal step beside it.

Workload: the nonlinear model (dx=2, dz=8, dy=8; growth-model outer block,
tanh-coupled inner block, z + 0.05 x^2 observed), N=4096 outer particles x
M=256 inner particles per outer particle, synthetic seeded observations.
A step is one look-ahead DPF step (Fig. 4: look-ahead weights, outer
resampling, new particles, inner resampling, propagation, inner measurement
update, estimates) with the observations already resident in HBM; the K
timed steps run as a captured HIP graph of the run's steps after the first (dpf_run).

In a run the new-cloud kernel of each step also computes the next step's
look-ahead weights, and a step-end kernel takes the estimates and prepares
the next step's resampling, so a step after the first is two kernels.

Prints one JSON line: inner-particle updates/s over the K timed steps (the
median of R timed repetitions of the K steps), the RMSE of the x estimate
against the simulated truth, the roofline of the dominant kernel (the
new-cloud kernel of a run, timed with HIP events that the library records on
its own stream around its launches): its algorithmic HBM bytes per launch
over its duration against the 8 TB/s peak, with its algorithmic VALU issue
slots beside it (the kernel is bound by vector-ALU issue, not by memory),
the FP64 oracle timed on a bounded sample on the host (all cores, and one),
and the learned proposal (trained on look-ahead pairs, then run at the same
N and M): its updates/s and RMSE beside the look-ahead step's on the same
fresh sequences.  Beside them: the linear-Gaussian model at the Kalman
filter's accuracy (the smallest N x M whose x estimate stays within a tenth
of a posterior standard deviation of the exact posterior mean), the
look-ahead, plain and learned steps at a fixed RMSE (32 fresh sequences as
32 filters of one handle), the batched run of 1024 ragged filters and the
high-dimensional inner block (dz = 64, N = 16384, M = 1024).
"""
import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "inner-particle updates/s at fixed RMSE vs Kalman/oracle; learned vs plain look-ahead"
UNIT = "inner-particle updates/s"
HBM_PEAK_GBS = 8000.0
N_OUT, M_IN, T_TRAJ = 4096, 256, 200
DX, DZ, DY = 2, 8, 8
PARAM_SEED, DATA_SEED, FILTER_SEED = 1, 2024, 7
LEARNED_PAIRS, LEARNED_EPOCHS = 1_000_000, 10
EVAL_SEQS, EVAL_SEED, ESS_FRAC = 8, 5000, 0.1
BATCH_F, BATCH_SEED = 1024, 7
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_nonlin_N4096_M256.txt")
KERNEL_SOURCES = ["dpf_kernels.hpp", "dpf_models.hpp", "dpf_rng.hpp", "dpf_seg.hpp"]

# Algorithmic bytes per inner particle of the new-cloud kernel of a run
# (FP32 state, dz = DZ): read the parent's ell (4) and lam (4) and the
# gathered z (4 dz); write z (4 dz), lam (4) and the next step's ell (4).
BYTES_PER_UPDATE = 8 * DZ + 16
# and per outer particle: read the ancestor's weight group (4) and x (4 dx);
# write x (4 dx), the ancestor and candidate (8), the cloud's partial sum
# (4 dz) and the next log-weight (4).
BYTES_PER_OUTER = 4 + 8 * DX + 8 + 4 * DZ + 4

# Algorithmic VALU issue slots per inner particle of the same kernel (one
# slot: one 32-bit lane operation; 32x32->64 products and transcendentals
# issue at quarter rate on CDNA and count 4).  A Philox4x32-10 block is ten
# rounds of two products and four exclusive ors; a U24 uniform is shift,
# convert, FMA; a remnant uniform four more to gather its bits; a Box-Muller
# pair is log, sqrt, cos, sin and three products.
PHILOX_BLOCK = 10 * (2 * 4 + 4)
BM_PAIR = 4 * 4 + 3


def normals_slots(n):
    """Issue slots for the first n standard normals of a draw in the packed
    layout (ten per two Philox blocks, the last two of each ten from the
    blocks' remnant uniforms)."""
    q, r = divmod(n, 10)
    blocks = 2 * q + (r > 0) + (r > 4)
    remnant = 2 * q + max(0, r - 8)
    return blocks * PHILOX_BLOCK + n * 3 + remnant * 4 + ((n + 1) // 2) * BM_PAIR


ISSUE_PER_UPDATE = {
    # this step: NEW_Z normals, f^z (two FMAs per component), log p(y|z)
    # (subtract and FMA per component), the inner resampling search (eight
    # FP64 compare-and-select steps), eq:qbar and the weighted moments
    "new_z": normals_slots(DZ),
    "propagate_and_weigh": 2 * DZ + 2 * DY + 2 + 8 * 3 + 4 + 2 + 3 * DZ,
    # the next step's look-ahead weight: the candidate's draw (x's normals,
    # then z's), f^x (growth
    # term: two products, add, reciprocal, FMAs), f^z's tanh(W x) (two FMAs,
    # exp and reciprocal, three more), f^z, the observation residual and
    # log p(y|x, z), ell = lam + that, and the running log-sum-exp
    "la_normals": normals_slots(DX + DZ),
    "la_model": DX * 10 + DZ * (2 * DX + 2 * 4 + 4) + 2 * DZ + DY + 2 * DY + 2 + 1 + 4 + 4,
}
VALU_SLOTS_PER_UPDATE = sum(ISSUE_PER_UPDATE.values())
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz: one lane slot per lane per clock
# (wave64 instructions take four clocks; packed FP32 is not used).
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def kernel_source_digest():
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1203_2394_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(phase):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None if it is missing or was taken on different kernel sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_digest") != kernel_source_digest():
        return None
    key = "%s_hbm_bytes_per_launch" % phase
    return float(kv[key]) if key in kv else None


def cpu_baseline_child(steps):
    """Time the FP64 oracle on `steps` look-ahead steps of the same workload."""
    import numpy as np

    import dpf_synth as S
    from oracle import ladpf
    from oracle.models import make_model

    spec = S.nonlin_c2(PARAM_SEED)
    model = make_model(spec.kind, spec.dx, spec.dz, spec.dy, spec.blob)
    _, _, ys = S.simulate(spec, steps, DATA_SEED)
    st = ladpf.init_state(model, N_OUT, M_IN, FILTER_SEED, 0)
    w0 = time.time()
    t0 = time.perf_counter()
    for t in range(steps):
        st, _ = ladpf.step(model, st, ys[t], FILTER_SEED, 0)
    dt = time.perf_counter() - t0
    print(json.dumps({"seconds": dt, "steps": steps, "updates": N_OUT * M_IN * steps,
                      "start": w0, "end": w0 + dt}))


def _cpu_children(n_proc, steps):
    """Run n_proc single-threaded oracle processes at once (each the same
    look-ahead workload); returns (wall seconds, total updates) or None."""
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        env[k] = "1"
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-baseline-child", str(steps)]
    procs = [subprocess.Popen(cmd, env=env, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)
             for _ in range(n_proc)]
    updates = 0
    starts, ends = [], []
    ok = True
    for pr in procs:
        out, err = pr.communicate(timeout=900)
        if pr.returncode != 0:
            sys.stderr.write(err)
            ok = False
            continue
        r = json.loads(out.strip().splitlines()[-1])
        updates += r["updates"]
        starts.append(r["start"])
        ends.append(r["end"])
    # the window from the first process's first step to the last one's end
    # (process start-up and the oracle's initialisation are not counted)
    return (max(ends) - min(starts), updates) if ok else None


def cpu_cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def run_cpu_baseline(steps):
    """The FP64 oracle on the host: one process per available core (at most
    16, the host share of one GPU) each taking `steps` look-ahead steps of the
    workload, and one process alone."""
    one = _cpu_children(1, steps)
    if one is None:
        return None
    n_proc = max(1, min(16, cpu_cores()))
    allc = _cpu_children(n_proc, steps) if n_proc > 1 else one
    if allc is None:
        return None
    wall, upd = allc
    return {"value": upd / wall, "unit": UNIT, "cores": n_proc, "kind": "oracle",
            "sample": "%d independent processes at once, each %d look-ahead steps of the same workload "
                      "(N=%d, M=%d), FP64 NumPy oracle, one thread each, %.1f s from the first step to the last; %d cores available "
                      "(os.cpu_count() %s)" % (n_proc, steps, N_OUT, M_IN, wall, cpu_cores(), os.cpu_count()),
            "single_core_value": one[1] / one[0]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--repeats", type=int, default=10,
                    help="timed repetitions of the K steps (the reported time is their median)")
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-proposal comparison")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched ragged-filter run")
    ap.add_argument("--no-highdim", action="store_true", help="skip the high-dimensional inner block run")
    ap.add_argument("--no-table1", action="store_true", help="skip the runs of the models of Table 1")
    ap.add_argument("--no-fixed-rmse", action="store_true",
                    help="skip the fixed-RMSE comparison of the look-ahead, plain and learned steps")
    ap.add_argument("--cpu-baseline-child", type=int, default=0)
    ap.add_argument("--only-run", action="store_true",
                    help="only the look-ahead runs (timed graph replays and the eager run with phase "
                         "events): every new-cloud launch is then a run's, for profiling")
    ap.add_argument("--only-highdim", action="store_true",
                    help="only the high-dimensional inner block run (for profiling)")
    ap.add_argument("--only-mlp", action="store_true",
                    help="only learned steps and training steps of an untrained network (for profiling the "
                         "network kernels)")
    ap.add_argument("--no-kalman", action="store_true",
                    help="skip the linear-Gaussian model at the Kalman filter's accuracy")
    ap.add_argument("--no-bandit", action="store_true",
                    help="skip the automatic decomposition experiment (Hedge / Exp3)")
    ap.add_argument("--only-bandit", action="store_true", help="only the automatic decomposition experiment")
    ap.add_argument("--only-nested", action="store_true",
                    help="only a nested look-ahead run (model 1 of Table 1, 256 x N=200 x M=20, K=8; profiling)")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="after the timed steps, run one device-to-device copy of this many MB "
                         "(a kernel of known traffic for calibrating hardware byte counters)")
    args = ap.parse_args()
    if args.cpu_baseline_child:
        cpu_baseline_child(args.cpu_baseline_child)
        return 0
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build measures the single-GPU step "
              "(multi-GPU sharding is described in DESIGN.md, not built); use --gpus 1", file=sys.stderr)
        return 2

    import ctypes

    import numpy as np
    import torch

    import dpf_synth as S
    import paper_1203_2394_amd as dpf

    K, W, R = args.steps, args.warmup, max(1, args.repeats)
    dev = torch.device("cuda:0")
    if args.only_highdim:
        print(json.dumps({"highdim": run_highdim(S, dpf, torch, np, dev)}))
        return 0
    if args.only_mlp:
        print(json.dumps({"mlp_profile": run_mlp_profile(S, dpf, torch, np, dev)}))
        return 0
    if args.only_bandit:
        print(json.dumps({"bandit": run_bandit(S, dpf, torch, np, dev)}))
        return 0
    if args.only_nested:
        print(json.dumps({"nested": run_nested_point(S, dpf, torch, np, dev)}))
        return 0
    spec = S.nonlin_c2(PARAM_SEED)
    n_obs = max(T_TRAJ, K, W)
    xs, _, ys = S.simulate(spec, n_obs, DATA_SEED)
    Y = torch.tensor(ys, dtype=torch.float32, device=dev).contiguous()
    f = dpf.Filter(spec.kind, spec.dx, spec.dz, spec.dy, spec.blob, [N_OUT], [M_IN], seed=FILTER_SEED,
                   device=dev)
    L = dpf.lib()
    h = f._h
    yptr = [ctypes.c_void_p(Y[t].data_ptr()) for t in range(n_obs)]
    updates = N_OUT * M_IN

    rmse_x = None
    if not args.only_run:
        # accuracy pass (not timed): one trajectory, RMSE of the x estimate vs truth
        xt, _ = f.run(Y[:T_TRAJ].reshape(T_TRAJ, 1, DY), use_graph=True)
        torch.cuda.synchronize()
        rmse_x = round(float(np.sqrt(np.mean(np.sum((xt[:, 0].cpu().numpy() - xs[1:T_TRAJ + 1]) ** 2,
                                                    axis=1)))), 4)
        # warm-up
        f.reset()
        for t in range(W):
            assert L.dpf_lookahead_step(h, yptr[t], None) == 0
    else:
        f.run(Y[:max(W, 2)].reshape(max(W, 2), 1, DY).contiguous(), trace=False, use_graph=False)
    # the K timed steps: replays of a captured chunk of steps, R timed
    # repetitions from the same initial state (the first run captures)
    f.reset()
    Yk = Y[:K].reshape(K, 1, DY).contiguous()
    f.run(Yk, trace=False, use_graph=True)  # capture
    runs = []
    for _ in range(R):
        f.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f.run(Yk, trace=False, use_graph=True)
        torch.cuda.synchronize()
        runs.append(time.perf_counter() - t0)
    dt = float(np.median(runs))

    # the same K steps as individual calls (no graph)
    edt = None
    if not args.only_run:
        f.reset()
        torch.cuda.synchronize()
        e0 = time.perf_counter()
        for t in range(K):
            if L.dpf_lookahead_step(h, yptr[t], None) != 0:
                raise RuntimeError(L.dpf_last_error().decode())
        torch.cuda.synchronize()
        edt = time.perf_counter() - e0

    # phase times of the same run executed eagerly: events the library
    # records on its stream between its launches (steps after the first:
    # the weights and statistics phases are empty there)
    f.reset()
    events = [torch.cuda.Event(enable_timing=True) for _ in range(5 * K)]
    f.set_phase_events(events)
    f.run(Yk, trace=False, use_graph=False)
    torch.cuda.synchronize()
    f.set_phase_events(None)
    phases = ["weights", "resample", "newcloud", "estimate"]
    ph_ms = {p: 0.0 for p in phases}
    for s in range(1, K):
        for i, p in enumerate(phases):
            ph_ms[p] += events[5 * s + i].elapsed_time(events[5 * s + i + 1]) / (K - 1)
    first_ms = {p: round(events[i].elapsed_time(events[i + 1]), 5) for i, p in enumerate(phases)}

    if args.copy_mb:
        n = args.copy_mb * (1 << 20) // 4
        src_t = torch.ones(n, dtype=torch.float32, device=dev)
        dst_t = torch.empty_like(src_t)
        torch.cuda.synchronize()
        dst_t.copy_(src_t)
        torch.cuda.synchronize()

    dur = ph_ms["newcloud"] * 1e-3
    slots_launch = updates * VALU_SLOTS_PER_UPDATE
    achieved = slots_launch / dur / 1e12
    bytes_launch = updates * BYTES_PER_UPDATE + N_OUT * BYTES_PER_OUTER
    gbs = bytes_launch / dur / 1e9
    roofline = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": read_traffic("newcloud"),
                "kernel": "k_newcloud (run: also the next step's look-ahead weights)",
                "bytes_per_update": BYTES_PER_UPDATE, "bytes_per_outer": BYTES_PER_OUTER,
                "bytes_per_launch": bytes_launch, "avg_ms": round(ph_ms["newcloud"], 5),
                "valu_view": {"op": "32-bit VALU lane issue slot (quarter-rate instructions count 4)",
                              "slots_per_update": VALU_SLOTS_PER_UPDATE, "slots_per_launch": slots_launch,
                              "achieved_tops": round(achieved, 2), "peak_tops": round(VALU_PEAK_TOPS, 2),
                              "frac": round(achieved / VALU_PEAK_TOPS, 4)}}
    f.close()

    learned, mlp = None, None
    if not (args.no_learned or args.only_run):
        mlp, learned = run_learned(S, dpf, torch, np, dev, K, W)
    fixed = None
    if not (args.no_fixed_rmse or args.only_run):
        fixed = run_fixed_rmse(S, dpf, torch, np, dev, mlp)
    batched = None if (args.no_batched or args.only_run) else run_batched(S, dpf, torch, np, dev)
    highdim = None if (args.no_highdim or args.only_run) else run_highdim(S, dpf, torch, np, dev)
    table1 = None
    if not (args.no_table1 or args.only_run):
        table1 = {"model1": run_table1(S, dpf, torch, np, dev, S.twodim_table1(), "Table 1 model 1"),
                  "model2": run_table1(S, dpf, torch, np, dev, S.fourdim_table1(), "Table 1 model 2")}
        table1["grid"] = run_table1_grid(S, dpf, torch, np, dev, table1)
    kalman = None if (args.no_kalman or args.only_run) else run_kalman_target(S, dpf, torch, np, dev)
    bandit = None if (args.no_bandit or args.only_run) else run_bandit(S, dpf, torch, np, dev)
    cpu = None if (args.no_cpu_baseline or args.only_run) else run_cpu_baseline(args.cpu_steps)
    out = {
        "metric": METRIC,
        "value": updates * K / dt,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "repeats": R,
        "ms_per_step": dt * 1e3 / K,
        "ms_per_step_runs": {"min": round(min(runs) * 1e3 / K, 5), "median": round(dt * 1e3 / K, 5),
                             "max": round(max(runs) * 1e3 / K, 5)},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "look-ahead DPF step, nonlinear model dx=2 dz=8 dy=8, N=4096 outer x M=256 inner",
                   "algo": "lookahead", "N": N_OUT, "M": M_IN, "dx": DX, "dz": DZ, "dy": DY,
                   "execution": "one captured HIP graph of the steps after the first (dpf_run); each step's "
                                "new-cloud kernel also computes the next step's look-ahead weights",
                   "rmse_x_T200": rmse_x},
        "eager_value": updates * K / edt if edt else None,
        "eager": "the K steps as separate dpf_lookahead_step calls (weights kernel every step, no graph)",
        "phase_ms": {p: round(v, 5) for p, v in ph_ms.items()},
        "first_step_phase_ms": first_ms,
        "roofline": roofline,
        "learned": learned,
        "fixed_rmse": fixed,
        "batched": batched,
        "highdim": highdim,
        "table1": table1,
        "kalman_target": kalman,
        "bandit": bandit,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    return 0


# the linear-Gaussian model at the Kalman filter's accuracy: sequences, their
# length, the (N, M) grid (visited in order of N x M) and the target on the
# time-averaged |x_hat - mu_KF| / sqrt(P_KF)
KF_SEQS, KF_T, KF_SEED = 16, 50, 31000
KF_GRID_N = (25, 50, 100, 200, 400, 800, 1600, 3200)
KF_GRID_M = (8, 16, 32, 50, 100)
KF_TARGET = 0.1


def kalman_x_posterior(blob, ys):
    """Exact filtered mean and variance of x_t given y_1..y_t for the
    linear-Gaussian model (dx = 1, dz = 2, dy = 1; parameter blob as the
    library takes it), by the Kalman filter on the joint state s = [x; z]:
    x' = Ax x + Cxz z + v, z' = Az z + Bzx x' + w, y = Hx x + Hz z + e, with
    x' substituted into z' and the prior s_0 ~ N(0, I).  The accuracy target
    of the measurement, not part of the filter's path."""
    import numpy as np
    b = np.asarray(blob, dtype=np.float64)
    Ax, Cxz, qx = b[0], b[1:3], b[3]
    Az, Bzx, qz = b[4:8].reshape(2, 2), b[8:10], b[10]
    Hx, Hz, r = b[11], b[12:14], b[14]
    F = np.zeros((3, 3))
    F[0, 0], F[0, 1:] = Ax, Cxz
    F[1:, 0] = Bzx * Ax
    F[1:, 1:] = Az + np.outer(Bzx, Cxz)
    G = np.zeros((3, 3))
    G[0, 0] = 1.0
    G[1:, 0] = Bzx
    G[1:, 1:] = np.eye(2)
    Q = G @ np.diag([qx, qz, qz]) @ G.T
    H = np.r_[Hx, Hz]
    mu, P = np.zeros(3), np.eye(3)
    means, var = [], []
    for y in np.asarray(ys, dtype=np.float64).reshape(-1):
        mu = F @ mu
        P = F @ P @ F.T + Q
        S_ = H @ P @ H + r
        K = P @ H / S_
        mu = mu + K * (y - H @ mu)
        P = P - np.outer(K, H @ P)
        P = 0.5 * (P + P.T)
        means.append(mu[0])
        var.append(P[0, 0])
    return np.asarray(means), np.asarray(var)


def run_kalman_target(S, dpf, torch, np, dev):
    """The linear-Gaussian model (dx=1, dz=2, dy=1) against its exact
    posterior: KF_SEQS fresh sequences of KF_T steps run as filters of one
    handle.  For the look-ahead and the plain step: the normalised error
    e = mean over sequences and steps of |x_hat_t - mu_t| / sqrt(P_t) at the
    nominal size (N = 100, M = 50), and the smallest N x M on the grid with
    e <= KF_TARGET, with its updates/s (graph-replayed run of the KF_SEQS
    filters, timed as a second run)."""
    spec = S.lingauss_c1(False)
    sims = [S.simulate(spec, KF_T, KF_SEED + q) for q in range(KF_SEQS)]
    ys = np.stack([sm[2] for sm in sims], axis=1)  # [T][F][1]
    Y = torch.tensor(ys, dtype=torch.float32, device=dev).contiguous()
    post = [kalman_x_posterior(spec.blob, ys[:, q, 0]) for q in range(KF_SEQS)]
    mu = np.stack([p_[0] for p_ in post], axis=1)
    sd = np.sqrt(np.stack([p_[1] for p_ in post], axis=1))

    def measure(algo, N, M, timed):
        f = dpf.Filter(spec.kind, spec.dx, spec.dz, spec.dy, spec.blob, [N] * KF_SEQS, [M] * KF_SEQS,
                       seed=FILTER_SEED, device=dev, algo=algo)
        xt, _ = f.run(Y, use_graph=True)
        e = float(np.mean(np.abs(xt.cpu().numpy()[:, :, 0] - mu) / sd))
        r = {"N": N, "M": M, "err": round(e, 4)}
        if timed:
            f.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            f.run(Y, trace=False, use_graph=True)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            r["updates_per_s"] = N * M * KF_SEQS * KF_T / dt
            r["ms_per_step"] = round(dt * 1e3 / KF_T, 4)
        f.close()
        return r

    grid = sorted(((n, m) for n in KF_GRID_N for m in KF_GRID_M), key=lambda v: (v[0] * v[1], v[0]))
    out = {"rule": "%d fresh sequences x T=%d as %d filters of one handle; e = mean over sequences and steps of "
                   "|x_hat - mu_KF| / sqrt(P_KF); smallest N x M on N in %s, M in %s with e <= %.2f"
                   % (KF_SEQS, KF_T, KF_SEQS, list(KF_GRID_N), list(KF_GRID_M), KF_TARGET)}
    for algo in ("lookahead", "plain"):
        res = {"at_N100_M50": measure(algo, 100, 50, True)}
        chosen = None
        for N, M in grid:
            r = measure(algo, N, M, False)
            if r["err"] <= KF_TARGET:
                chosen = measure(algo, N, M, True)
                break
        res["at_target"] = chosen if chosen is not None else {"reached": False}
        out[algo] = res
    return out


def run_mlp_profile(S, dpf, torch, np, dev):
    """Learned steps (network, inner pass, decision, commit) and training
    steps of an untrained network on the nonlinear model at N = 4096,
    M = 256: a short, fixed sequence of the network kernels for counter
    passes."""
    from paper_1203_2394_amd import proposal as PR

    spec = S.nonlin_c2(PARAM_SEED)
    g = np.random.default_rng(0)
    B = 4096
    X = torch.tensor(g.normal(size=(B, 26)), dtype=torch.float32, device=dev)
    xt = torch.tensor(g.normal(size=(B, 2)), dtype=torch.float32, device=dev)
    mlp, _ = PR.train(X, xt, epochs=2, batch=B, lr=1e-3, seed=0)
    _, _, ys = S.simulate(spec, 8, DATA_SEED)
    Y = torch.tensor(ys, dtype=torch.float32, device=dev).reshape(8, 1, DY).contiguous()
    f = dpf.Filter(spec.kind, spec.dx, spec.dz, spec.dy, spec.blob, [N_OUT], [M_IN], seed=FILTER_SEED,
                   device=dev)
    f.set_proposal(mlp, ess_frac=0.0)
    for t in range(8):
        f.learned_step(Y[t])
    torch.cuda.synchronize()
    f.close()
    return {"learned_steps": 8, "training_steps": 2, "batch": B}


# the decomposition experiment of Section 4.3: sequences, horizon, change
# point, filter sizes, reward and bandit parameters, the RMSE window
BD_SEQS, BD_T, BD_TC, BD_N, BD_M, BD_SEED = 16, 4000, 600, 200, 20, 50000
BD_ALPHA, BD_GAMMA, BD_ETA, BD_WINDOW = 1e-3, 0.2, 0.5, (3000, 4000)
BD_CHECKPOINTS = (1, 100, 300, 600, 700, 1000, 1500, 2000, 3000, 4000)


def run_bandit(S, dpf, torch, np, dev):
    """Automatic decomposition (Section 3, Section 4.3): model 1 of Table 1
    with its transition laws swapped from t = BD_TC on, BD_SEQS fresh
    sequences of BD_T steps.  Action 1 samples x first, action 2 z first:
    each is a look-ahead DPF over all sequences (one handle, filters =
    sequences, N x M particles, graph-replayed run) that forms the predicted
    observation of every step.  Rewards r = alpha / (alpha + (y - yhat)^2);
    Hedge (every action's reward) and Exp3 (the chosen action's only) pick
    at each step which filter's estimate is reported, with a seeded stream
    per sequence.  Reports the action probabilities over time (means over
    the sequences) and the RMSE of x and z over the window for each fixed
    action, Hedge and Exp3."""
    from paper_1203_2394_amd import bandit as BB

    T = BD_T
    specs = [S.twodim_table1(tswap=BD_TC), S.twodim_table1(tswap=BD_TC, zfirst=True)]
    sims = [S.simulate(specs[0], T, BD_SEED + q) for q in range(BD_SEQS)]
    Y = torch.tensor(np.stack([sm[2] for sm in sims], axis=1), dtype=torch.float32, device=dev).contiguous()
    tx = np.stack([sm[0][1:, 0] for sm in sims], axis=1)  # [T][F]
    tz = np.stack([sm[1][1:, 0] for sm in sims], axis=1)
    y = Y[:, :, 0].cpu().numpy().astype(np.float64)
    est, yhat, timing = [], [], []
    for a, spec in enumerate(specs):
        f = dpf.Filter(spec.kind, spec.dx, spec.dz, spec.dy, spec.blob, [BD_N] * BD_SEQS, [BD_M] * BD_SEQS,
                       seed=FILTER_SEED + a, device=dev)
        tr = f.set_prediction(True, trace_T=T)
        xt, zt = f.run(Y, use_graph=True)
        o, i = xt[:, :, 0].cpu().numpy(), zt[:, :, 0].cpu().numpy()
        est.append((o, i) if a == 0 else (i, o))          # (x_hat, z_hat) in the paper's variables
        yhat.append(tr.cpu().numpy().astype(np.float64))
        f.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f.run(Y, trace=False, use_graph=True)
        torch.cuda.synchronize()
        timing.append(time.perf_counter() - t0)
        f.close()
    R = np.stack([BB.reward(y - yh, BD_ALPHA) for yh in yhat], axis=2)   # [T][F][2]
    R = np.where(np.isfinite(R), R, 0.0)
    lo, hi = BD_WINDOW
    w = slice(lo, hi)  # rows t-1 for lo < t <= hi

    def rmse(xh, zh):
        ex = (xh[w] - tx[w]) ** 2
        ez = (zh[w] - tz[w]) ** 2
        return {"x": round(float(np.sqrt(np.nanmean(ex))), 4), "z": round(float(np.sqrt(np.nanmean(ez))), 4)}

    out = {"action1_x_first": rmse(*est[0]), "action2_z_first": rmse(*est[1])}
    probs = {}
    for name in ("hedge", "exp3"):
        acts = np.empty((T, BD_SEQS), dtype=np.int64)
        p2 = np.empty((T, BD_SEQS))
        for q in range(BD_SEQS):
            u = BB.uniforms(BD_SEED + 7 * q + (1 if name == "exp3" else 0), T)
            if name == "hedge":
                a_, P = BB.run_hedge(R[:, q], BD_ETA, u)
                p2[:, q] = P[:, 1]
            else:
                a_, P, Ph = BB.run_exp3(R[:, q], BD_ETA, BD_GAMMA, u)
                p2[:, q] = Ph[:, 1]
            acts[:, q] = a_
        xh = np.where(acts == 0, est[0][0], est[1][0])
        zh = np.where(acts == 0, est[0][1], est[1][1])
        out[name] = rmse(xh, zh)
        out[name]["last100_action2_frac"] = round(float(np.mean(acts[-100:] == 1)), 4)
        probs[name] = {str(c): round(float(np.mean(p2[c - 1])), 4) for c in BD_CHECKPOINTS}
    upd = BD_N * BD_M * BD_SEQS * T
    return {"rmse_window": "%d < t <= %d" % (lo, hi), "rmse": out,
            "p_action2_mean": probs,
            "updates_per_s": {"action1_x_first": upd / timing[0], "action2_z_first": upd / timing[1]},
            "config": {"workload": "model 1 of Table 1 with its transitions swapped from t=%d, %d sequences x "
                                   "T=%d as filters of one handle per decomposition, N=%d, M=%d" % (
                                       BD_TC, BD_SEQS, T, BD_N, BD_M),
                       "reward": "alpha/(alpha+eps^2), alpha=%g" % BD_ALPHA, "gamma": BD_GAMMA, "eta": BD_ETA,
                       "execution": "both decompositions run every step (graph-replayed runs); the bandit "
                                    "chooses which filter's estimate is reported"}}


HD_N, HD_M, HD_T, HD_SEED = 16384, 1024, 100, 4

# fixed-RMSE comparison: sequences, their length, the outer-particle grid and
# the tolerance on the reference RMSE (the look-ahead step at N = 4096)
FR_SEQS, FR_SEED, FR_T = 32, 9000, 200
FR_GRID = (256, 512, 1024, 2048, 4096, 8192)
FR_TOL = 1.05


def run_fixed_rmse(S, dpf, torch, np, dev, mlp):
    """Throughput at a fixed RMSE (look-ahead, plain and learned steps on the
    nonlinear model, M = 256), in the serving shape: FR_SEQS fresh sequences
    of FR_T steps run as FR_SEQS filters of one handle (one graph-replayed
    run).  The reference RMSE (x_hat against the simulated truth, root of the
    mean over steps and sequences) is the look-ahead run's at N = 4096.  For
    each method: RMSE and updates/s at N = 4096, and the smallest N on
    FR_GRID whose RMSE is within FR_TOL of the reference with its updates/s
    and outer particle-steps/s.  Each run is timed as a second run of the
    same handle (reset, cached graph)."""
    spec = S.nonlin_c2(PARAM_SEED)
    sims = [S.simulate(spec, FR_T, FR_SEED + q) for q in range(FR_SEQS)]
    Y = torch.tensor(np.stack([sm[2] for sm in sims], axis=1), dtype=torch.float32, device=dev).contiguous()
    truth = np.stack([sm[0][1:FR_T + 1] for sm in sims], axis=1)  # [T][F][dx]

    def measure(algo, N):
        f = dpf.Filter(spec.kind, spec.dx, spec.dz, spec.dy, spec.blob, [N] * FR_SEQS, [M_IN] * FR_SEQS,
                       seed=FILTER_SEED, device=dev, algo="plain" if algo == "plain" else "lookahead")
        learned = algo == "learned"
        if learned:
            f.set_proposal(mlp, ess_frac=ESS_FRAC)
        xt, _ = f.run(Y, use_graph=True, learned=learned)
        err = np.sum((xt.cpu().numpy() - truth) ** 2, axis=2)
        f.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f.run(Y, use_graph=True, learned=learned)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        f.close()
        steps = FR_SEQS * FR_T
        per_seq = np.sqrt(err.mean(axis=0))
        return {"N": N, "rmse_x": round(float(np.sqrt(err.mean())), 5),
                "seq_rmse_median": round(float(np.median(per_seq)), 4), "seq_rmse_max": round(float(per_seq.max()), 4),
                "updates_per_s": N * M_IN * steps / dt, "particle_steps_per_s": N * steps / dt,
                "ms_per_step": dt * 1e3 / FR_T}

    methods = ["lookahead", "plain"] + (["learned"] if mlp is not None else [])
    at_ref = {m: measure(m, N_OUT) for m in methods}
    ref = at_ref["lookahead"]["rmse_x"]
    target = FR_TOL * ref
    out = {"reference_rmse_x": ref, "target_rmse_x": round(target, 5),
           "rule": "%d fresh sequences x T=%d as %d filters of one handle (M=%d); reference: look-ahead RMSE "
                   "at N=%d; per method the smallest N in %s with RMSE <= %.2f x reference"
                   % (FR_SEQS, FR_T, FR_SEQS, M_IN, N_OUT, list(FR_GRID), FR_TOL),
           "at_N%d" % N_OUT: at_ref, "at_target": {}}
    for m in methods:
        chosen = None
        for N in FR_GRID:
            r = at_ref[m] if N == N_OUT else measure(m, N)
            if r["rmse_x"] <= target:
                chosen = r
                break
        out["at_target"][m] = chosen if chosen is not None else {"reached": False}
    return out


TD_SEQS, TD_T, TD_N, TD_M, TD_SEED = 32, 250, 4096, 256, 12000


def run_table1(S, dpf, torch, np, dev, spec, name):
    """A model of Table 1 (time-varying drifts): TD_SEQS fresh sequences of
    TD_T steps as filters of one handle (N = 4096, M = 256), look-ahead and
    plain runs, graph-replayed; updates/s of the second run of each handle
    and the RMSE of x_hat and z_hat."""
    sims = [S.simulate(spec, TD_T, TD_SEED + q) for q in range(TD_SEQS)]
    Y = torch.tensor(np.stack([sm[2] for sm in sims], axis=1), dtype=torch.float32, device=dev).contiguous()
    tx = np.stack([sm[0][1:] for sm in sims], axis=1)
    tz = np.stack([sm[1][1:] for sm in sims], axis=1)
    out = {"config": {"workload": "%s (dx=%d dz=%d dy=%d), %d sequences x T=%d as filters of one handle, "
                                  "N=%d, M=%d" % (name, spec.dx, spec.dz, spec.dy, TD_SEQS, TD_T, TD_N, TD_M)}}
    for algo in ("lookahead", "plain"):
        f = dpf.Filter(spec.kind, spec.dx, spec.dz, spec.dy, spec.blob, [TD_N] * TD_SEQS, [TD_M] * TD_SEQS,
                       seed=FILTER_SEED, device=dev, algo=algo)
        xt, zt = f.run(Y, use_graph=True)
        ex = np.sqrt(np.mean((xt.cpu().numpy() - tx) ** 2, axis=(0, 2)))
        ez = np.sqrt(np.mean((zt.cpu().numpy() - tz) ** 2, axis=(0, 2)))
        f.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f.run(Y, trace=False, use_graph=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        f.close()
        out[algo] = {"updates_per_s": TD_N * TD_M * TD_SEQS * TD_T / dt, "ms_per_step": dt * 1e3 / TD_T,
                     "rmse_x": round(float(np.sqrt(np.mean(ex ** 2))), 4),
                     "rmse_z": round(float(np.sqrt(np.mean(ez ** 2))), 4),
                     "seq_rmse_x_median": round(float(np.median(ex)), 4),
                     "seq_rmse_x_max": round(float(ex.max()), 4)}
    return out


GRID_SEQS, GRID_N, GRID_M, GRID_SEED = 256, (20, 50, 100, 200), (10, 20), 20000
GRID_K = (1, 4, 8)  # companions per look-ahead candidate (nested estimator)


def run_nested_point(S, dpf, torch, np, dev, N=200, M=20, K=8):
    """One point of the Table 1 grid with the nested look-ahead estimator:
    model 1, GRID_SEQS sequences of TD_T steps as filters of one handle, run
    twice (the second timed)."""
    spec = S.twodim_table1()
    sims = [S.simulate(spec, TD_T, GRID_SEED + q) for q in range(GRID_SEQS)]
    Y = torch.tensor(np.stack([sm[2] for sm in sims], axis=1), dtype=torch.float32, device=dev).contiguous()
    f = dpf.Filter(spec.kind, spec.dx, spec.dz, spec.dy, spec.blob, [N] * GRID_SEQS, [M] * GRID_SEQS,
                   seed=FILTER_SEED, device=dev)
    f.set_companions(K)
    f.run(Y, trace=False, use_graph=True)
    f.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f.run(Y, trace=False, use_graph=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    f.close()
    return {"N": N, "M": M, "K": K, "filters": GRID_SEQS, "T": TD_T, "ms_per_step": round(dt * 1e3 / TD_T, 4),
            "updates_per_s": N * M * GRID_SEQS * TD_T / dt}


def run_table1_grid(S, dpf, torch, np, dev, ref):
    """Section 4.1's study on the models of Table 1: RMSE of x_hat and z_hat
    and the fraction of diverged runs against (N, M) for the look-ahead step
    (with its plain and its Rao-Blackwellised x estimate), the look-ahead
    step with the nested estimator (K companions per candidate, K in
    GRID_K) and the plain step, GRID_SEQS fresh 250-step sequences per point
    run as filters of one handle.  A run diverges when an estimate is
    non-finite or its RMSE of x exceeds 3x the reference (the look-ahead run
    at N = 4096, M = 256 of `ref`)."""
    out = {}
    for key, spec in (("model1", S.twodim_table1()), ("model2", S.fourdim_table1())):
        sims = [S.simulate(spec, TD_T, GRID_SEED + q) for q in range(GRID_SEQS)]
        Y = torch.tensor(np.stack([sm[2] for sm in sims], axis=1), dtype=torch.float32, device=dev).contiguous()
        tx = np.stack([sm[0][1:] for sm in sims], axis=1)
        tz = np.stack([sm[1][1:] for sm in sims], axis=1)
        lim = 3.0 * ref[key]["lookahead"]["rmse_x"]
        rows = []
        for N in GRID_N:
            for M in GRID_M:
                row = {"N": N, "M": M}
                for algo in ("lookahead", "plain") + tuple("K%d" % k for k in GRID_K):
                    f = dpf.Filter(spec.kind, spec.dx, spec.dz, spec.dy, spec.blob, [N] * GRID_SEQS,
                                   [M] * GRID_SEQS, seed=FILTER_SEED, device=dev,
                                   algo="plain" if algo == "plain" else "lookahead")
                    arms = {}
                    if algo == "plain":
                        xt, zt = f.run(Y, use_graph=True)
                        arms["plain"] = (xt, zt)
                    elif algo.startswith("K"):
                        f.set_companions(int(algo[1:]))
                        xt, zt = f.run(Y, use_graph=True)
                        arms["lookahead_" + algo] = (xt, zt)
                    else:
                        # step calls (a run gives the same bits) so that the
                        # Rao-Blackwellised estimate can follow every step
                        xs, zs, rs = [], [], []
                        for t in range(TD_T):
                            f.lookahead_step(Y[t])
                            e = f.estimate()
                            xs.append(e["xhat"])
                            zs.append(e["zhat"])
                            rs.append(f.estimate_rb())
                        zt = torch.stack(zs)
                        arms["lookahead"] = (torch.stack(xs), zt)
                        arms["lookahead_rb"] = (torch.stack(rs), zt)
                    # the arm's own time: a second run of the handle, graph-replayed
                    f.reset()
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    f.run(Y, trace=False, use_graph=True)
                    torch.cuda.synchronize()
                    ms = (time.perf_counter() - t0) * 1e3 / TD_T
                    f.close()
                    for arm, (xt, zt) in arms.items():
                        xt, zt = xt.cpu().numpy(), zt.cpu().numpy()
                        ex = np.sqrt(np.mean((xt - tx) ** 2, axis=(0, 2)))
                        ez = np.sqrt(np.mean((zt - tz) ** 2, axis=(0, 2)))
                        div = ~np.isfinite(ex) | ~np.isfinite(ez) | (ex > lim)
                        ok = ~div
                        row[arm] = {"rmse_x": round(float(np.sqrt(np.mean(ex[ok] ** 2))), 4) if ok.any() else None,
                                    "rmse_z": round(float(np.sqrt(np.mean(ez[ok] ** 2))), 4) if ok.any() else None,
                                    "diverged": round(float(div.mean()), 4), "ms_per_step": round(ms, 4)}
                rows.append(row)
        out[key] = {"divergence_limit_rmse_x": round(lim, 4), "points": rows}
    out["config"] = {"workload": "models 1 and 2 of Table 1, %d fresh sequences x T=%d per point as filters of "
                                 "one handle, N in %s, M in %s" % (GRID_SEQS, TD_T, list(GRID_N), list(GRID_M)),
                     "rmse": "over the sequences that did not diverge",
                     "ms_per_step": "graph-replayed run of the %d filters (the Rao-Blackwellised arm is its "
                                    "look-ahead arm's estimate, same run)" % GRID_SEQS,
                     "arms": "lookahead (one companion per candidate, paired), lookahead_rb (its "
                             "Rao-Blackwellised x estimate), lookahead_K<k> (nested estimator, k companions per "
                             "candidate), plain"}
    return out


def run_highdim(S, dpf, torch, np, dev):
    """The high-dimensional inner block (dx=4, dz=64, dy=32; banded A,
    B sin(x), 32x64 projection, Gaussian / Student-t(3) outlier mixture
    likelihood), N=16384 x M=1024 (16.8M inner particles, 4.3 GB per state
    copy), one look-ahead run of HD_T steps, graph-replayed, timed after an
    untimed run that records the estimates (RMSE against the simulated truth)
    and an untimed run of the timed run's own graph."""
    spec = S.highdim_c4(PARAM_SEED)
    xs, zs, ys = S.simulate(spec, HD_T, HD_SEED)
    Y = torch.tensor(ys, dtype=torch.float32, device=dev).reshape(HD_T, 1, spec.dy).contiguous()
    f = dpf.Filter(spec.kind, spec.dx, spec.dz, spec.dy, spec.blob, [HD_N], [HD_M], seed=FILTER_SEED,
                   device=dev)
    # untimed run with the estimates: RMSE of x and z against the simulated truth
    xt, zt = f.run(Y, trace=True, use_graph=True)
    torch.cuda.synchronize()
    ex = xt[:, 0].cpu().numpy().astype(np.float64) - np.asarray(xs[1:HD_T + 1])
    ez = zt[:, 0].cpu().numpy().astype(np.float64) - np.asarray(zs[1:HD_T + 1])
    rmse = {"x": round(float(np.sqrt(np.mean(np.sum(ex ** 2, axis=1)))), 4),
            "z": round(float(np.sqrt(np.mean(np.sum(ez ** 2, axis=1)))), 4),
            "rule": "root of the mean over the %d steps of the squared Euclidean error of x_hat (z_hat)" % HD_T}
    f.reset()
    f.run(Y, trace=False, use_graph=True)  # the timed run's own graph, captured untimed
    f.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f.run(Y, trace=False, use_graph=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    updates = HD_N * HD_M
    ms = dt * 1e3 / HD_T
    # algorithmic bytes of a run step: z read (gathered) and written (4 dz
    # each), lam, the parent's ell and the next ell (4 each)
    bytes_step = updates * (8 * spec.dz + 16)
    f.close()
    return {"value": updates * HD_T / dt, "unit": UNIT, "ms_per_step": round(ms, 4), "steps": HD_T, "rmse": rmse,
            "config": {"workload": "look-ahead DPF, high-dimensional inner block dx=4 dz=64 dy=32 "
                                   "(Student-t outlier mixture), N=16384 outer x M=1024 inner",
                       "execution": "dpf_run, graph replays"},
            "hbm_view": {"bytes_per_step": bytes_step, "achieved_gbs": round(bytes_step / (ms * 1e-3) / 1e9, 1),
                         "frac": round(bytes_step / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}}


def run_batched(S, dpf, torch, np, dev):
    """1024 independent filters of the linear-Gaussian model with ragged N, M
    and horizons T_f in one handle, run to the end as graph replays; tile
    classes for each inner size from the autotuner, and the default tiling
    beside it."""
    from paper_1203_2394_amd import autotune as AT

    spec = S.lingauss_c1(False)
    rb = S.ragged_batch(F=BATCH_F, seed=BATCH_SEED)
    F, T = BATCH_F, int(rb.T.max())
    ys = np.zeros((T, F, spec.dy), dtype=np.float32)
    for q in range(F):
        ys[:rb.T[q], q] = S.simulate(spec, int(rb.T[q]), int(rb.data_seeds[q]))[2]
    Y = torch.tensor(ys, device=dev)
    Tf = torch.tensor(rb.T, dtype=torch.int32, device=dev)
    updates = float(np.sum(rb.N.astype(np.float64) * rb.M * rb.T))
    t0 = time.perf_counter()
    table = AT.tune(spec, np.unique(rb.M), N=1024, steps=16, reps=2, simulate=S.simulate, device=dev)
    tune_s = time.perf_counter() - t0
    out = {}
    for mode in ("default", "tuned"):
        f = dpf.Filter(spec.kind, spec.dx, spec.dz, spec.dy, spec.blob, rb.N, rb.M, seed=BATCH_SEED, device=dev)
        if mode == "tuned":
            f.set_tiling(AT.classes_for(table, rb.M))
        f.run(Y, Tf=Tf, trace=False, use_graph=True)  # capture and warm up
        f.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f.run(Y, Tf=Tf, trace=False, use_graph=True)
        torch.cuda.synchronize()
        out[mode] = time.perf_counter() - t0
        f.close()
    cls = dpf.tile_classes()
    return {
        "value": updates / out["tuned"],
        "unit": UNIT,
        "seconds": round(out["tuned"], 4),
        "default_tiling_value": updates / out["default"],
        "inner_updates": updates,
        "config": {"workload": "F=%d linear-Gaussian filters (dx=1 dz=2 dy=1), N log-uniform in [256, 4096], "
                               "M in {32, 64, 128}, T in [50, 500], one handle, graph replays" % F,
                   "sum_N": int(rb.N.sum()), "sum_NM": int(np.sum(rb.N.astype(np.int64) * rb.M)),
                   "T_max": T},
        "tiling": {str(m): {"class": v["class"], "seg_jpt": cls[v["class"]],
                            "ms_per_step": {str(k): round(t, 4) for k, t in v["ms"].items()}}
                   for m, v in table.items()},
        "tune_s": round(tune_s, 2),
    }


def run_learned(S, dpf, torch, np, dev, K, W):
    """The learned proposal on the same workload: train on pairs from the
    look-ahead DPF (fresh sequences), compare RMSE with the look-ahead step on
    fresh evaluation sequences at the same N and M, time K learned steps."""
    from paper_1203_2394_amd import proposal as PR

    spec = S.nonlin_c2(PARAM_SEED)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    X, xt = PR.generate_pairs(spec, LEARNED_PAIRS, simulate=S.simulate, device=dev)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    mlp, losses = PR.train(X, xt, epochs=LEARNED_EPOCHS, batch=4096, lr=1e-3, seed=0)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    ev = PR.evaluate(spec, mlp, N=N_OUT, M=M_IN, T=T_TRAJ, n_seq=EVAL_SEQS, data_seed=EVAL_SEED,
                     ess_frac=ESS_FRAC, simulate=S.simulate, device=dev, timing_reps=1)

    # K timed learned steps, graph-replayed like the look-ahead steps
    xs, _, ys = S.simulate(spec, max(K, W), DATA_SEED)
    Yk = torch.tensor(ys[:K], dtype=torch.float32, device=dev).reshape(K, 1, DY).contiguous()
    f = dpf.Filter(spec.kind, spec.dx, spec.dz, spec.dy, spec.blob, [N_OUT], [M_IN], seed=FILTER_SEED,
                   device=dev)
    f.set_proposal(mlp, ess_frac=ESS_FRAC)
    f.run(Yk, trace=False, use_graph=True, learned=True)  # capture
    f.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f.run(Yk, trace=False, use_graph=True, learned=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    f.reset()
    torch.cuda.synchronize()
    e0 = time.perf_counter()
    for t in range(K):
        f.learned_step(Yk[t])
    torch.cuda.synchronize()
    edt = time.perf_counter() - e0
    f.close()
    updates = N_OUT * M_IN
    return mlp, {
        "value": updates * K / dt,
        "ms_per_step": dt * 1e3 / K,
        "eager_value": updates * K / edt,
        "rmse_x": round(ev["learned"]["rmse_x"], 4),
        "rmse_x_lookahead": round(ev["lookahead"]["rmse_x"], 4),
        "rmse_ratio": round(ev["learned"]["rmse_x"] / ev["lookahead"]["rmse_x"], 4),
        "fallback_frac": round(ev["learned"]["fallback_frac"], 4),
        "eval": "%d fresh sequences x T=%d, N=%d, M=%d, fallback when ESS < %.2g N" % (
            EVAL_SEQS, T_TRAJ, N_OUT, M_IN, ESS_FRAC),
        "train": {"pairs": LEARNED_PAIRS, "epochs": LEARNED_EPOCHS, "batch": 4096, "lr": 1e-3,
                  "nll_first_epoch": round(losses[0], 4), "nll_last_epoch": round(losses[-1], 4),
                  "generate_s": round(gen_s, 3), "train_s": round(train_s, 3)},
        "dtype": "bf16 network (MFMA, FP32 accumulate), f32 filter",
    }


if __name__ == "__main__":
    sys.exit(main())
