"""The nested look-ahead estimator (Fig. 4 step 1 with K companions per
candidate, eq:weightsMC) on the GPU against the oracle: the look-ahead
weights themselves (a mismatch must be explained by a companion ancestor's
near tie), then the rest of the step (outer resampling, candidate draw,
inner resampling and propagation) against the oracle's steps 3-4 on the
GPU's weights; runs equal step calls bit for bit."""
import math

import numpy as np
import pytest

import dpf_synth as S
import paper_1203_2394_amd as dpf
from oracle import ladpf
from oracle.models import make_model

from parity_util import TOL, assert_clean, compare_la, compare_nested_weights, to_state32

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


SPECS = {
    "lingauss": lambda: S.lingauss_c1(False),
    "lingauss_coupled": lambda: S.lingauss_c1(True),
    "nonlin": lambda: S.nonlin_c2(1),
    "highdim": lambda: S.highdim_c4(1),
    "twodim": lambda: S.twodim_table1(),
    "fourdim": lambda: S.fourdim_table1(),
}


@pytest.mark.parametrize("name,N,M,K,warm,steps,cls", [
    ("lingauss", 103, 50, 3, 2, 2, None),
    ("lingauss_coupled", 64, 37, 4, 2, 2, None),
    ("lingauss_coupled", 9, 300, 3, 1, 1, None),     # a 256-lane segment per particle
    ("nonlin", 150, 64, 2, 1, 2, None),
    ("nonlin", 20, 300, 5, 1, 1, None),
    ("highdim", 6, 256, 2, 1, 1, None),
    ("twodim", 100, 10, 8, 3, 2, None),
    ("twodim", 60, 20, 4, 5, 2, None),
    ("twodim", 7, 300, 2, 2, 1, None),
    ("fourdim", 90, 20, 8, 3, 2, None),
    ("fourdim", 40, 128, 1, 2, 1, None),
    # 16-lane segments: (16, 2), (16, 4), (16, 8)
    ("twodim", 61, 20, 8, 3, 2, 11),
    ("lingauss_coupled", 42, 50, 3, 2, 1, 12),
    ("nonlin", 50, 100, 2, 1, 1, 13),
])
def test_nested_step_parity(name, N, M, K, warm, steps, cls):
    spec = SPECS[name]()
    model = make_model(spec.kind, spec.dx, spec.dz, spec.dy, spec.blob)
    seed = 6161
    _, _, ys = S.simulate(spec, warm + steps, 13)
    ys = ys.astype(np.float32).astype(np.float64)
    st = ladpf.init_state(model, N, M, seed, 0)
    for t in range(warm):
        st, _ = ladpf.step(model, st, ys[t], seed, 0, n_comp=K)
    f = dpf.Filter(spec.kind, spec.dx, spec.dz, spec.dy, spec.blob, [N], [M], seed=seed)
    if cls is not None:
        f.set_tiling([cls])
    f.set_companions(K)
    predict = spec.dy == 1
    if predict:
        f.set_prediction(True)
    for t in range(warm, warm + steps):
        st32 = to_state32(st)
        f.import_state(torch.from_numpy(f.pack_state(st32["t"], st32["x"], st32["z"], st32["lam"])))
        f.lookahead_step(torch.tensor(ys[t], dtype=torch.float32))
        g = f.unpack_state(f.export_state())
        ell = f.copy_buffer(dpf.BUF_ELL).cpu().numpy().reshape(N, M).astype(np.float64)
        logw = f.copy_buffer(dpf.BUF_LOGW).cpu().numpy()
        anc = f.copy_buffer(dpf.BUF_ANC).cpu().numpy()
        sel = f.copy_buffer(dpf.BUF_SEL).cpu().numpy()
        est = f.estimate()
        # (a) the nested weights against the oracle's own
        rw, ell_o, tainted = compare_nested_weights(model, st32, ys[t], seed, 0, K, ell)
        print("nested weights %s N=%d M=%d K=%d t=%d: %s" % (name, N, M, K, t + 1, rw.line()), flush=True)
        assert rw["ell_unexplained"] == 0, rw.line()
        assert rw["err_ell"] <= TOL, rw.line()
        assert rw["tainted_rows"] <= max(1, N // 50), rw.line()
        # (b) steps 3-4 against the oracle's on the GPU's weights
        gs = {"x": g["x"][0], "z": g["z"][0], "lam": g["lam"][0]}
        r, st, info = compare_la(model, st32, ys[t], seed, 0, gs, ell, logw, anc, sel, ell_given=ell)
        print("nested step %s N=%d M=%d K=%d t=%d: %s" % (name, N, M, K, t + 1, r.line()), flush=True)
        assert_clean(r, n=N)
        ll = float(est["loglik"][0])
        assert abs(ll - info["dlogz"]) <= 1e-4 * max(1.0, abs(info["dlogz"])), (ll, info["dlogz"])
        ess = float(est["ess"][0])
        assert abs(ess - info["ess"]) <= 1e-4 * info["ess"], (ess, info["ess"])
        if predict and rw["tainted_rows"] == 0:
            # the predicted observation over the companions
            _, _, _, _, hmean = ladpf.lookahead_nested(model, st32, ys[t], seed, 0, K)
            yo = float(ladpf.predicted_observation(st32["lam"], hmean)[0])
            yg = float(f.predicted_observation()[0])
            assert abs(yg - yo) <= 1e-4 * max(1.0, abs(yo)), (yg, yo)


@pytest.mark.parametrize("name,N,M,K", [("nonlin", [300, 90], [64, 40], 3), ("twodim", [200, 50], [20, 10], 4)])
def test_nested_run_equals_step_calls(name, N, M, K):
    """A run with companions takes every step whole; graph replays, eager
    run and step calls give the same bits, across a chunk boundary."""
    spec = SPECS[name]()
    T = 19
    Y = np.stack([S.simulate(spec, T, 70 + q)[2] for q in range(len(N))], axis=1).astype(np.float32)
    a = dpf.Filter(spec.kind, spec.dx, spec.dz, spec.dy, spec.blob, N, M, seed=21)
    a.set_companions(K)
    for t in range(T):
        a.lookahead_step(torch.from_numpy(Y[t]))
    ref = a.export_state().cpu().numpy()
    for use_graph in (True, False):
        b = dpf.Filter(spec.kind, spec.dx, spec.dz, spec.dy, spec.blob, N, M, seed=21)
        b.set_companions(K)
        b.run(torch.from_numpy(Y), use_graph=use_graph)
        assert np.array_equal(ref, b.export_state().cpu().numpy()), use_graph
        assert torch.equal(a.estimate()["loglik"], b.estimate()["loglik"])
        for buf in (dpf.BUF_ELL, dpf.BUF_LOGW):
            assert torch.equal(a.copy_buffer(buf), b.copy_buffer(buf)), buf
    # back to the paired form: the same handle continues with the fused run
    b.set_companions(0)
    b.reset()
    c = dpf.Filter(spec.kind, spec.dx, spec.dz, spec.dy, spec.blob, N, M, seed=21)
    b.run(torch.from_numpy(Y), use_graph=True)
    c.run(torch.from_numpy(Y), use_graph=True)
    assert np.array_equal(b.export_state().cpu().numpy(), c.export_state().cpu().numpy())


def test_companion_count_is_validated():
    spec = SPECS["nonlin"]()
    f = dpf.Filter(spec.kind, spec.dx, spec.dz, spec.dy, spec.blob, [16], [8], seed=1)
    for bad in (-1, 1025):
        with pytest.raises(dpf.DPFError):
            f.set_companions(bad)
    p = dpf.Filter(spec.kind, spec.dx, spec.dz, spec.dy, spec.blob, [16], [8], seed=1, algo="plain")
    with pytest.raises(dpf.DPFError):
        p.set_companions(2)
