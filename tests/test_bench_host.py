"""Host-side pieces of bench.py (no GPU): the single-GPU guard, the CPU
baseline leg (the oracle on one step of the workload), the issue-slot count
behind the roofline, and that the committed counter summary was taken on the
current kernel sources (else the bench reports its traffic as null)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _run(*args, timeout=300):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + list(args), capture_output=True,
                          text=True, timeout=timeout)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run("--gpus", "2", timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_cpu_baseline_child_times_the_oracle_on_the_workload():
    r = _run("--cpu-baseline-child", "1")
    assert r.returncode == 0, r.stderr
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["steps"] == 1 and out["updates"] == bench.N_OUT * bench.M_IN == 4096 * 256
    assert out["seconds"] > 0


def test_issue_slot_count():
    # Philox4x32-10 block: ten rounds of two quarter-rate 32x32->64 products
    # (4 slots each) and four exclusive ors; a Box-Muller pair: four
    # quarter-rate transcendentals and three full-rate operations
    assert bench.PHILOX_BLOCK == 120 and bench.BM_PAIR == 19
    # n normals in the packed layout: two blocks per ten normals (one for a
    # remainder of up to four, two above), three slots per uniform, four more
    # per remnant uniform, one Box-Muller pair per two normals
    assert bench.normals_slots(8) == 2 * 120 + 24 + 4 * 19
    assert bench.normals_slots(2) == 120 + 6 + 19
    assert bench.normals_slots(10) == 2 * 120 + 30 + 2 * 4 + 5 * 19
    assert bench.normals_slots(3) == 120 + 9 + 2 * 19
    assert bench.normals_slots(64) == 13 * 120 + 192 + 12 * 4 + 32 * 19
    # nonlinear model: the new z (8 normals) and the candidate's x and z (10)
    assert bench.ISSUE_PER_UPDATE["new_z"] == bench.normals_slots(8)
    assert bench.ISSUE_PER_UPDATE["la_normals"] == bench.normals_slots(10)
    assert bench.VALU_SLOTS_PER_UPDATE == sum(bench.ISSUE_PER_UPDATE.values()) == 1000
    assert abs(bench.VALU_PEAK_TOPS - 39.3216) < 1e-9


def test_traffic_summary_matches_the_kernel_sources():
    assert bench.read_traffic("newcloud") is not None
    assert bench.read_traffic("post") is not None


def test_cpu_baseline_reports_all_cores_and_one():
    r = bench.run_cpu_baseline(1)
    assert r is not None and r["kind"] == "oracle"
    assert r["cores"] == max(1, min(16, bench.cpu_cores()))
    assert r["value"] > 0 and r["single_core_value"] > 0
    assert "processes" in r["sample"]


def test_bench_kalman_posterior_equals_the_oracle_kalman_filter():
    """The accuracy target the bench measures against is the exact posterior:
    its x marginal must equal the oracle's joint Kalman filter."""
    import numpy as np

    import dpf_synth as S
    from oracle.kalman import kalman_filter
    from oracle.models import make_model

    spec = S.lingauss_c1(False)
    _, _, ys = S.simulate(spec, 40, 3)
    mu, var = bench.kalman_x_posterior(spec.blob, ys[:, 0])
    m = make_model(spec.kind, spec.dx, spec.dz, spec.dy, spec.blob)
    means, covs, _ = kalman_filter(m, ys)
    assert np.allclose(mu, means[:, 0], rtol=1e-12, atol=1e-12)
    assert np.allclose(var, covs[:, 0, 0], rtol=1e-12, atol=1e-12)
