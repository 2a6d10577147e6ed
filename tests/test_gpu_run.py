"""Multi-step runs on the GPU: many ragged filters in one handle against the
oracle, graph replay against plain step calls (bit for bit), resume from an
exported state, per-filter horizons, and the data-dependent flags."""
import numpy as np
import pytest

import dpf_synth as S
import paper_1203_2394_amd as dpf
from oracle import ladpf
from oracle.models import make_model

from parity_util import assert_clean, compare_la, to_state32

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _filter(spec, N, M, seed=11, algo="lookahead"):
    return dpf.Filter(spec.kind, spec.dx, spec.dz, spec.dy, spec.blob, N, M, seed=seed, algo=algo)


def test_ragged_batch_matches_oracle_per_filter():
    """One handle, filters of uneven N and M (every tile class), each compared
    with the oracle run under its own filter index."""
    spec = S.lingauss_c1(True)
    model = make_model(spec.kind, spec.dx, spec.dz, spec.dy, spec.blob)
    N = [37, 150, 70, 33, 5, 12]
    M = [32, 64, 100, 300, 1500, 1]
    F, seed = len(N), 2024
    ys = np.stack([S.simulate(spec, 3, 50 + f)[2] for f in range(F)], axis=1)  # [T][F][1]
    ys = ys.astype(np.float32).astype(np.float64)
    states = []
    for f in range(F):
        st = ladpf.init_state(model, N[f], M[f], seed, f)
        st, _ = ladpf.step(model, st, ys[0, f], seed, f)
        states.append(to_state32(st))
    g = _filter(spec, N, M, seed)
    g.import_state(torch.from_numpy(g.pack_state([s["t"] for s in states], [s["x"] for s in states],
                                                 [s["z"] for s in states], [s["lam"] for s in states])))
    g.lookahead_step(torch.tensor(ys[1], dtype=torch.float32))
    rb = g.estimate_rb().cpu().numpy()
    out = g.unpack_state(g.export_state())
    ell = g.copy_buffer(dpf.BUF_ELL).cpu().numpy()
    logw = g.copy_buffer(dpf.BUF_LOGW).cpu().numpy()
    anc = g.copy_buffer(dpf.BUF_ANC).cpu().numpy()
    sel = g.copy_buffer(dpf.BUF_SEL).cpu().numpy()
    oo = io = 0
    for f in range(F):
        n, m = N[f], M[f]
        gs = {"x": out["x"][f], "z": out["z"][f], "lam": out["lam"][f]}
        r, _, info = compare_la(model, states[f], ys[1, f], seed, f, gs, ell[io:io + n * m].reshape(n, m),
                                logw[oo:oo + n], anc[oo:oo + n], sel[oo:oo + n])
        print("filter %d N=%d M=%d: %s" % (f, n, m, r.line()), flush=True)
        assert_clean(r, max_flip_frac=0.05, n=n)
        # the Rao-Blackwellised estimate of each filter of the ragged handle
        assert np.allclose(rb[f], info["xhat_rb"], rtol=1e-4, atol=1e-3), (f, rb[f], info["xhat_rb"])
        oo += n
        io += n * m


@pytest.mark.parametrize("N,M", [([300, 64], [256, 50]), ([5000, 40], [24, 130]), ([16700, 40], [8, 24])])
def test_graph_run_equals_step_calls_bit_for_bit(N, M):
    """A run (fused steps, graph replays or eager) against step calls; N = 5000
    has 20 resampling groups, N = 16700 66 (more than 64 groups in a handle:
    the step end runs as two launches)."""
    spec = S.nonlin_c2(1)
    T = 6
    Y = np.stack([S.simulate(spec, T, 9 + f)[2] for f in range(2)], axis=1).astype(np.float32)
    a = _filter(spec, N, M)
    for t in range(T):
        a.lookahead_step(torch.from_numpy(Y[t]))
    sa = a.export_state().cpu().numpy()
    ea = a.estimate()
    b = _filter(spec, N, M)
    xt, zt = b.run(torch.from_numpy(Y), use_graph=True)
    sb = b.export_state().cpu().numpy()
    eb = b.estimate()
    assert np.array_equal(sa, sb)
    assert torch.equal(ea["xhat"], eb["xhat"]) and torch.equal(ea["loglik"], eb["loglik"])
    assert torch.equal(xt[-1], eb["xhat"])
    # a look-ahead run computes each step's weights in the previous step's
    # new-cloud kernel: the last step's weights must be the step calls' ones
    for buf in (dpf.BUF_ELL, dpf.BUF_LOGW, dpf.BUF_ANC, dpf.BUF_SEL):
        assert torch.equal(a.copy_buffer(buf), b.copy_buffer(buf)), buf
    c = _filter(spec, N, M)
    c.run(torch.from_numpy(Y), use_graph=False)
    assert np.array_equal(sa, c.export_state().cpu().numpy())
    for buf in (dpf.BUF_ELL, dpf.BUF_LOGW):
        assert torch.equal(a.copy_buffer(buf), c.copy_buffer(buf)), buf
    # and a step call after a run continues from the same state
    a.lookahead_step(torch.from_numpy(Y[T - 1]))
    b.lookahead_step(torch.from_numpy(Y[T - 1]))
    assert np.array_equal(a.export_state().cpu().numpy(), b.export_state().cpu().numpy())
    assert torch.equal(a.copy_buffer(dpf.BUF_ELL), b.copy_buffer(dpf.BUF_ELL))


@pytest.mark.parametrize("T", [17, 20, 300, 514])
def test_run_chunks_and_remainder_equal_step_calls(T):
    """Look-ahead runs as graphs: the first step eager, then one captured
    graph of the other T - 1 steps (T - 1 <= 256), or replays of a 256-step
    chunk and a captured tail of the remaining steps (T = 300: one chunk and
    43 steps; T = 514: two chunks and one step) -- the alternating weight
    buffers must line up across every boundary.  A second run of the same
    length replays the cached graphs."""
    spec = S.nonlin_c2(1)
    N, M = [200, 90], [64, 40]
    Y = np.stack([S.simulate(spec, T, 41 + f)[2] for f in range(2)], axis=1).astype(np.float32)
    a = _filter(spec, N, M)
    for t in range(T):
        a.lookahead_step(torch.from_numpy(Y[t]))
    sa = a.export_state().cpu().numpy()
    ea = a.estimate()
    b = _filter(spec, N, M)
    for rep in range(2):
        b.reset()
        xt, _ = b.run(torch.from_numpy(Y), use_graph=True)
        assert np.array_equal(sa, b.export_state().cpu().numpy()), rep
        eb = b.estimate()
        assert torch.equal(ea["xhat"], eb["xhat"]) and torch.equal(ea["loglik"], eb["loglik"])
        for buf in (dpf.BUF_ELL, dpf.BUF_LOGW):
            assert torch.equal(a.copy_buffer(buf), b.copy_buffer(buf)), (rep, buf)


def test_rb_estimate_follows_step_calls_only():
    """dpf_estimate_rb after a look-ahead step; NaN for a filter that sat the
    step out; refused after a run (the estimate needs the step's own buffers
    and state copies)."""
    spec = S.nonlin_c2(1)
    Y = np.stack([S.simulate(spec, 3, 71 + f)[2] for f in range(2)], axis=1).astype(np.float32)
    f = _filter(spec, [300, 90], [64, 40])
    f.lookahead_step(torch.from_numpy(Y[0]))
    rb = f.estimate_rb().cpu().numpy()
    assert np.all(np.isfinite(rb))
    f.lookahead_step(torch.from_numpy(Y[1]), active=np.array([1, 0], dtype=np.uint8))
    rb = f.estimate_rb().cpu().numpy()
    assert np.all(np.isfinite(rb[0])) and np.all(np.isnan(rb[1]))
    f.run(torch.from_numpy(Y), use_graph=False)
    with pytest.raises(dpf.DPFError):
        f.estimate_rb()


@pytest.mark.parametrize("model", ["twodim", "fourdim"])
@pytest.mark.parametrize("algo", ["lookahead", "plain"])
def test_time_varying_model_run_equals_step_calls(algo, model):
    """Models 1 and 2 of Table 1 have drifts that depend on t: a run (fused
    steps across a chunk boundary) and step calls must agree bit for bit."""
    spec = S.twodim_table1() if model == "twodim" else S.fourdim_table1()
    N, M, T = [300, 77], [64, 130], 19
    Y = np.stack([S.simulate(spec, T, 61 + f)[2] for f in range(2)], axis=1).astype(np.float32)
    a = _filter(spec, N, M, algo=algo)
    step = a.lookahead_step if algo == "lookahead" else a.step
    for t in range(T):
        step(torch.from_numpy(Y[t]))
    b = _filter(spec, N, M, algo=algo)
    xt, _ = b.run(torch.from_numpy(Y), use_graph=True)
    # (the plain DPF's state is the proposals x, z; its lam block is unused)
    sa, sb = a.unpack_state(a.export_state()), b.unpack_state(b.export_state())
    keys = ("t", "x", "z", "lam") if algo == "lookahead" else ("t", "x", "z")
    for k in keys:
        for u, v in zip(sa[k], sb[k]):
            assert np.array_equal(u, v), k
    assert torch.equal(a.estimate()["xhat"], b.estimate()["xhat"])
    assert torch.equal(a.estimate()["zhat"], b.estimate()["zhat"])
    assert np.all(np.isfinite(xt.cpu().numpy()))


@pytest.mark.parametrize("algo", ["lookahead", "plain"])
def test_wide_z_run_equals_step_calls(algo):
    """The high-dimensional model forms its residuals on the matrix cores with
    every lane of a wave taking part (zeros where a lane holds no inner
    particle), in the weights kernel and in the new-cloud kernel that computes
    the next step's weights in a run: run and step calls agree bit for bit,
    with 32-lane segments (two outer particles per wave, an odd N), inner
    sizes that leave lanes empty and a 256-lane class."""
    spec = S.highdim_c4(1)
    N, M, T = [33, 10, 3], [24, 100, 512], 4
    Y = np.stack([S.simulate(spec, T, 81 + f)[2] for f in range(3)], axis=1).astype(np.float32)
    a = _filter(spec, N, M, algo=algo)
    step = a.lookahead_step if algo == "lookahead" else a.step
    for t in range(T):
        step(torch.from_numpy(Y[t]))
    b = _filter(spec, N, M, algo=algo)
    xt, _ = b.run(torch.from_numpy(Y), use_graph=True)
    sa, sb = a.unpack_state(a.export_state()), b.unpack_state(b.export_state())
    keys = ("t", "x", "z", "lam") if algo == "lookahead" else ("t", "x", "z")
    for k in keys:
        for u, v in zip(sa[k], sb[k]):
            assert np.array_equal(u, v), k
    ea, eb = a.estimate(), b.estimate()
    assert torch.equal(ea["xhat"], eb["xhat"]) and torch.equal(ea["loglik"], eb["loglik"])
    assert np.all(np.isfinite(xt.cpu().numpy()))


@pytest.mark.parametrize("use_run", [False, True])
def test_step_end_kernels_agree(use_run):
    """Filter 0 alone (one step-end launch) and next to a filter of 66
    resampling groups (the step end as two launches): the same bits (every
    reduction of a filter runs in its own fixed order)."""
    spec = S.nonlin_c2(1)
    T = 4
    Y = np.stack([S.simulate(spec, T, 31 + f)[2] for f in range(2)], axis=1).astype(np.float32)
    outs = []
    for N, M in (([300], [256]), ([300, 16700], [256, 8])):
        f = _filter(spec, N, M)
        Yf = np.ascontiguousarray(Y[:, :len(N)])
        if use_run:
            f.run(torch.from_numpy(Yf), use_graph=False)
        else:
            for t in range(T):
                f.lookahead_step(torch.from_numpy(Yf[t]))
        st = f.unpack_state(f.export_state())
        est = f.estimate()
        outs.append((st["x"][0], st["z"][0], st["lam"][0], est["xhat"][0].cpu().numpy(),
                     est["zhat"][0].cpu().numpy(), float(est["loglik"][0])))
    for u, v in zip(outs[0], outs[1]):
        assert np.array_equal(u, v)


def test_per_filter_horizons_and_resume():
    spec = S.lingauss_c1()
    N, M, T = [64, 128, 32], [50, 64, 100], 8
    Tf = [8, 3, 5]
    Y = np.stack([S.simulate(spec, T, 20 + f)[2] for f in range(3)], axis=1).astype(np.float32)
    a = _filter(spec, N, M, seed=5)
    xt, _ = a.run(torch.from_numpy(Y), Tf=Tf, use_graph=True)
    s = a.unpack_state(a.export_state())
    assert list(s["t"]) == Tf
    xt = xt.cpu().numpy()
    for f in range(3):
        assert np.all(np.isfinite(xt[:Tf[f], f])) and np.all(np.isnan(xt[Tf[f]:, f]))
    # the same filters stepped one at a time with an activity mask
    b = _filter(spec, N, M, seed=5)
    for t in range(T):
        act = np.array([t < Tf[f] for f in range(3)], dtype=np.uint8)
        b.lookahead_step(torch.from_numpy(Y[t]), active=act)
    assert np.array_equal(a.export_state().cpu().numpy(), b.export_state().cpu().numpy())
    # resume: export after 4 steps, import into a fresh handle, continue
    c = _filter(spec, N, M, seed=5)
    for t in range(4):
        c.lookahead_step(torch.from_numpy(Y[t]))
    blob = c.export_state()
    d = _filter(spec, N, M, seed=5)
    d.import_state(blob)
    e = _filter(spec, N, M, seed=5)
    for t in range(6):
        e.lookahead_step(torch.from_numpy(Y[t]))
    for t in range(4, 6):
        d.lookahead_step(torch.from_numpy(Y[t]))
    assert np.array_equal(d.export_state().cpu().numpy(), e.export_state().cpu().numpy())


@pytest.mark.parametrize("algo", ["lookahead", "plain"])
def test_nonfinite_observation_sets_flags_and_keeps_state_finite(algo):
    spec = S.nonlin_c2(1)
    f = _filter(spec, [50, 60], [64, 32], algo=algo)
    y = np.zeros((2, 8), dtype=np.float32)
    y[1, 3] = np.nan
    step = f.lookahead_step if algo == "lookahead" else f.step
    step(torch.from_numpy(y))
    est = f.estimate()
    fl = est["flags"].cpu().numpy()
    assert fl[0] == 0
    assert fl[1] & dpf.FLAG_NONFINITE and fl[1] & dpf.FLAG_DEGENERATE_OUTER
    s = f.unpack_state(f.export_state())
    assert np.all(np.isfinite(s["x"][1])) and np.all(np.isfinite(s["z"][1]))
    # a later finite observation continues normally
    step(torch.from_numpy(np.zeros((2, 8), dtype=np.float32)))
    assert np.all(np.isfinite(f.estimate()["xhat"].cpu().numpy()))


def test_two_runs_are_bit_identical():
    spec = S.highdim_c4(1)
    N, M = [16], [1024]
    Y = S.simulate(spec, 3, 1)[2][:, None, :].astype(np.float32)
    outs = []
    for _ in range(2):
        f = _filter(spec, N, M, seed=3)
        f.run(torch.from_numpy(Y), use_graph=False)
        outs.append(f.export_state().cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


def test_autotuner_picks_a_measured_class_and_round_trips(tmp_path):
    from paper_1203_2394_amd import autotune as AT
    spec = S.lingauss_c1(False)
    table = AT.tune(spec, [32, 64, 128], N=256, steps=4, reps=1, simulate=S.simulate, n_filters=4)
    for M, v in table.items():
        assert v["class"] in AT.candidates(M)
        seg, jpt = dpf.tile_classes()[v["class"]]
        assert seg * jpt >= M
        assert all(t > 0 for t in v["ms"].values())
    path = str(tmp_path / "tiles.json")
    AT.save(table, path, spec)
    assert AT.load(path, spec) == table
    # a ragged handle with the tuned classes runs and matches the default
    # tiling statistically (same model, same sizes)
    N, M = [300, 200, 100], [32, 64, 128]
    f = _filter(spec, N, M, seed=5)
    f.set_tiling(AT.classes_for(table, M))
    ys = np.stack([S.simulate(spec, 20, 70 + q)[2] for q in range(3)], axis=1)
    xt, _ = f.run(torch.tensor(ys, dtype=torch.float32), use_graph=True)
    assert np.all(np.isfinite(xt.cpu().numpy()))


def _lingauss_tuned_handle(seed, cls):
    """Three linear-Gaussian filters (M = 32, 64, 128) under tile classes the
    autotuner picks for the batched run: the 16-lane (16, 2), (16, 4), (16, 8)
    or the 32-lane (32, 1), (32, 2), (32, 4)."""
    spec = S.lingauss_c1(False)
    N, M = [300, 200, 150], [32, 64, 128]
    f = _filter(spec, N, M, seed=seed)
    f.set_tiling(cls)
    return spec, N, M, f


@pytest.mark.parametrize("cls", [[11, 12, 13], [0, 6, 7]])
def test_tuned_batched_classes_match_oracle(cls):
    """The tile classes the autotuner picks for the batched linear-Gaussian
    run, in one ragged handle, two consecutive steps each compared with the
    oracle per filter (every step starts from the oracle's state, rounded)."""
    seed = 4040
    assert [dpf.tile_classes()[c][0] for c in cls] in ([16, 16, 16], [32, 32, 32])
    spec, N, M, g = _lingauss_tuned_handle(seed, cls)
    model = make_model(spec.kind, spec.dx, spec.dz, spec.dy, spec.blob)
    F = len(N)
    ys = np.stack([S.simulate(spec, 4, 90 + f)[2] for f in range(F)], axis=1)  # [T][F][1]
    ys = ys.astype(np.float32).astype(np.float64)
    states = []
    for f in range(F):
        st = ladpf.init_state(model, N[f], M[f], seed, f)
        st, _ = ladpf.step(model, st, ys[0, f], seed, f)
        states.append(to_state32(st))
    for t in (1, 2):
        g.import_state(torch.from_numpy(g.pack_state([s["t"] for s in states], [s["x"] for s in states],
                                                     [s["z"] for s in states], [s["lam"] for s in states])))
        g.lookahead_step(torch.tensor(ys[t], dtype=torch.float32))
        out = g.unpack_state(g.export_state())
        ell = g.copy_buffer(dpf.BUF_ELL).cpu().numpy()
        logw = g.copy_buffer(dpf.BUF_LOGW).cpu().numpy()
        anc = g.copy_buffer(dpf.BUF_ANC).cpu().numpy()
        sel = g.copy_buffer(dpf.BUF_SEL).cpu().numpy()
        est = g.estimate()
        oo = io = 0
        nxt = []
        for f in range(F):
            n, m = N[f], M[f]
            gs = {"x": out["x"][f], "z": out["z"][f], "lam": out["lam"][f]}
            r, new_o, info = compare_la(model, states[f], ys[t, f], seed, f, gs,
                                        ell[io:io + n * m].reshape(n, m), logw[oo:oo + n], anc[oo:oo + n],
                                        sel[oo:oo + n])
            print("tuned class step %d filter %d N=%d M=%d: %s" % (t, f, n, m, r.line()), flush=True)
            assert_clean(r, n=n)
            ll = float(est["loglik"][f])
            assert abs(ll - info["dlogz"]) <= 1e-4 * max(1.0, abs(info["dlogz"])), (f, ll, info["dlogz"])
            nxt.append(to_state32(new_o))
            oo += n
            io += n * m
        states = nxt


@pytest.mark.parametrize("cls", [[11, 12, 13], [0, 6, 7]])
def test_tuned_batched_classes_run_equals_step_calls(cls):
    """Under the same classes, a graph-replayed run (fused steps: each step's
    look-ahead weights inside the previous new-cloud launch) equals step
    calls bit for bit, with per-filter horizons across a chunk boundary."""
    T = 21
    spec, N, M, a = _lingauss_tuned_handle(77, cls)
    Y = np.stack([S.simulate(spec, T, 130 + f)[2] for f in range(len(N))], axis=1).astype(np.float32)
    Tf = [21, 18, 9]
    for t in range(T):
        act = np.array([t < Tf[f] for f in range(len(N))], dtype=np.uint8)
        a.lookahead_step(torch.from_numpy(Y[t]), active=act)
    _, _, _, b = _lingauss_tuned_handle(77, cls)
    b.run(torch.from_numpy(Y), Tf=Tf, use_graph=True)
    assert np.array_equal(a.export_state().cpu().numpy(), b.export_state().cpu().numpy())
    ea, eb = a.estimate(), b.estimate()
    for k in ("xhat", "zhat", "ess", "loglik"):
        assert torch.equal(ea[k], eb[k]), k


def test_cumulative_evidence_over_steps():
    """The cumulative evidence sums the per-step increments: two steps on the
    GPU from an imported state against the oracle's increments, the second
    taken by the oracle from the GPU's own state after the first (so index
    flips in the first step do not matter)."""
    spec = S.nonlin_c2(1)
    model = make_model(spec.kind, spec.dx, spec.dz, spec.dy, spec.blob)
    N, M, seed = 700, 64, 31
    _, _, ys = S.simulate(spec, 3, 12)
    ys = ys.astype(np.float32).astype(np.float64)
    st = ladpf.init_state(model, N, M, seed, 0)
    st, _ = ladpf.step(model, st, ys[0], seed, 0)
    st32 = to_state32(st)
    f = _filter(spec, [N], [M], seed=seed)
    f.import_state(torch.from_numpy(f.pack_state(st32["t"], st32["x"], st32["z"], st32["lam"])))
    f.lookahead_step(torch.tensor(ys[1], dtype=torch.float32))
    g1 = f.unpack_state(f.export_state())
    _, info1 = ladpf.step(model, st32, ys[1], seed, 0)
    f.lookahead_step(torch.tensor(ys[2], dtype=torch.float32))
    st_g = {"x": g1["x"][0].astype(np.float64), "z": g1["z"][0].astype(np.float64),
            "lam": g1["lam"][0].astype(np.float64), "t": int(g1["t"][0])}
    _, info2 = ladpf.step(model, st_g, ys[2], seed, 0)
    ll = float(f.estimate()["loglik"][0])
    ref = info1["dlogz"] + info2["dlogz"]
    print("cumulative evidence gpu %.9g oracle %.9g" % (ll, ref), flush=True)
    assert abs(ll - ref) <= 1e-4 * max(1.0, abs(ref))


@pytest.mark.parametrize("zfirst", [False, True])
def test_predicted_observation_run_equals_step_calls(zfirst):
    """The predicted observation of a fused run (each step's look-ahead draws
    formed in the previous step's new-cloud launch) equals step calls', bit
    for bit, per step, across a chunk boundary and a change point."""
    spec = S.twodim_table1(tswap=9, zfirst=zfirst)
    N, M, T = [300, 77], [64, 20], 21
    Y = np.stack([S.simulate(spec, T, 81 + q)[2] for q in range(2)], axis=1).astype(np.float32)
    a = _filter(spec, N, M)
    a.set_prediction(True)
    ys = []
    for t in range(T):
        a.lookahead_step(torch.from_numpy(Y[t]))
        ys.append(a.predicted_observation())
    ref = torch.stack(ys)
    b = _filter(spec, N, M)
    tr = b.set_prediction(True, trace_T=T)
    b.run(torch.from_numpy(Y), use_graph=True)
    assert np.array_equal(a.export_state().cpu().numpy(), b.export_state().cpu().numpy())
    assert torch.equal(ref, tr), (ref[:3], tr[:3])
    assert torch.equal(b.predicted_observation(), ref[-1])
    # switching the prediction off leaves the run's results unchanged
    c = _filter(spec, N, M)
    c.run(torch.from_numpy(Y), use_graph=True)
    assert np.array_equal(b.export_state().cpu().numpy(), c.export_state().cpu().numpy())
