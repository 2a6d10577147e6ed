#!/usr/bin/env python3
"""Throughput benchmark of the look-ahead DPF step on one MI355X.

Workload: the nonlinear model (dx=2, dz=8, dy=8; growth-model outer block,
tanh-coupled inner block, z + 0.05 x^2 observed), N=4096 outer particles x
M=256 inner particles per outer particle, synthetic seeded observations.
A step is one call of dpf_lookahead_step (Fig. 4: look-ahead weights, outer
resampling, new particles, inner resampling, propagation, inner measurement
update, estimates) with the observations already resident in HBM.

Prints one JSON line: inner-particle updates/s over the K timed steps, the
roofline of the dominant kernel (algorithmic bytes per launch over its
average duration, timed with HIP events recorded by the library on its own
stream), and the FP64 oracle timed on a bounded sample on the host.
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_nonlin_N4096_M256.txt")
KERNEL_SOURCES = ["dpf_kernels.hpp", "dpf_models.hpp", "dpf_rng.hpp", "dpf_seg.hpp"]

# Algorithmic bytes per inner particle of each phase (FP32 state, dz = DZ):
#   weights:   read z (4 dz) + lam (4), write ell (4)
#   new cloud: read parent ell (4) + lam (4) + gathered z (4 dz),
#              write z (4 dz) + lam (4)
BYTES_PER_UPDATE = {"weights": 4 * DZ + 8, "newcloud": 8 * DZ + 12}
# and per outer particle: weights reads x (4 dx) writes log w (4);
# new cloud reads the ancestor (4) and the parent x (4 dx), writes x (4 dx),
# the selected index (4) and the cloud's partial sum (4 dz).
BYTES_PER_OUTER = {"weights": 4 * DX + 4, "newcloud": 8 + 8 * DX + 4 * DZ}


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
    t0 = time.perf_counter()
    for t in range(steps):
        st, _ = ladpf.step(model, st, ys[t], FILTER_SEED, 0)
    dt = time.perf_counter() - t0
    print(json.dumps({"seconds": dt, "steps": steps, "updates": N_OUT * M_IN * steps}))


def run_cpu_baseline(steps):
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        env[k] = "1"
    out = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-child", str(steps)],
                         env=env, capture_output=True, text=True, timeout=600)
    if out.returncode != 0:
        sys.stderr.write(out.stderr)
        return None
    r = json.loads(out.stdout.strip().splitlines()[-1])
    return {"value": r["updates"] / r["seconds"], "unit": UNIT, "cores": 1, "kind": "oracle",
            "sample": "%d look-ahead steps of the same workload (N=%d, M=%d), FP64 NumPy oracle, "
                      "one thread, %.1f s" % (steps, N_OUT, M_IN, r["seconds"])}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-baseline-child", type=int, default=0)
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

    K, W = args.steps, args.warmup
    dev = torch.device("cuda:0")
    spec = S.nonlin_c2(PARAM_SEED)
    n_obs = max(T_TRAJ, K, W)
    xs, _, ys = S.simulate(spec, n_obs, DATA_SEED)
    Y = torch.tensor(ys, dtype=torch.float32, device=dev).contiguous()
    f = dpf.Filter(spec.kind, spec.dx, spec.dz, spec.dy, spec.blob, [N_OUT], [M_IN], seed=FILTER_SEED,
                   device=dev)
    L = dpf.lib()
    h = f._h
    yptr = [ctypes.c_void_p(Y[t].data_ptr()) for t in range(n_obs)]

    # accuracy pass (not timed): one trajectory, RMSE of the x estimate vs truth
    xt, _ = f.run(Y[:T_TRAJ].reshape(T_TRAJ, 1, DY), use_graph=True)
    torch.cuda.synchronize()
    rmse_x = float(np.sqrt(np.mean((xt[:, 0].cpu().numpy() - xs[1:T_TRAJ + 1]) ** 2)))

    f.reset()
    for t in range(W):
        assert L.dpf_lookahead_step(h, yptr[t], None) == 0
    f.reset()
    events = [torch.cuda.Event(enable_timing=True) for _ in range(5 * K)]
    f.set_phase_events(events)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(K):
        if L.dpf_lookahead_step(h, yptr[t], None) != 0:
            raise RuntimeError(L.dpf_last_error().decode())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    f.set_phase_events(None)
    phases = ["weights", "resample", "newcloud", "estimate"]
    ph_ms = {p: 0.0 for p in phases}
    for s in range(K):
        for i, p in enumerate(phases):
            ph_ms[p] += events[5 * s + i].elapsed_time(events[5 * s + i + 1]) / K

    # graph-replayed variant of the same K steps (one capture, K replays)
    f.reset()
    Yk = Y[:K].reshape(K, 1, DY).contiguous()
    f.run(Yk, trace=False, use_graph=True)  # capture + warm
    f.reset()
    torch.cuda.synchronize()
    g0 = time.perf_counter()
    f.run(Yk, trace=False, use_graph=True)
    torch.cuda.synchronize()
    gdt = time.perf_counter() - g0

    if args.copy_mb:
        n = args.copy_mb * (1 << 20) // 4
        src_t = torch.ones(n, dtype=torch.float32, device=dev)
        dst_t = torch.empty_like(src_t)
        torch.cuda.synchronize()
        dst_t.copy_(src_t)
        torch.cuda.synchronize()

    updates = N_OUT * M_IN
    dom = max(("weights", "newcloud"), key=lambda p: ph_ms[p])
    bytes_launch = updates * BYTES_PER_UPDATE[dom] + N_OUT * BYTES_PER_OUTER[dom]
    achieved = bytes_launch / (ph_ms[dom] * 1e-3) / 1e9
    traffic = read_traffic(dom)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "k_newcloud" if dom == "newcloud" else "k_la_weights",
                "bytes_per_launch": bytes_launch, "avg_ms": round(ph_ms[dom], 5)}
    cpu = None if args.no_cpu_baseline else run_cpu_baseline(args.cpu_steps)
    out = {
        "metric": METRIC,
        "value": updates * K / dt,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": dt * 1e3 / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "look-ahead DPF step, nonlinear model dx=2 dz=8 dy=8, N=4096 outer x M=256 inner",
                   "algo": "lookahead", "N": N_OUT, "M": M_IN, "dx": DX, "dz": DZ, "dy": DY,
                   "rmse_x_T200": round(rmse_x, 4)},
        "phase_ms": {p: round(v, 5) for p, v in ph_ms.items()},
        "graph_value": updates * K / gdt,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
