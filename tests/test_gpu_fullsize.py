"""Parity at the benchmark's full sizes, in the launch configuration the
benchmark times.

* High-dimensional inner block, one filter of N = 16384 outer x M = 1024
  inner particles (dz = 64, 4.3 GB per state copy), default tile class: the
  oracle cannot step the whole filter, so sampled outputs are compared one by
  one -- the look-ahead log-weights of sampled outer particles (from their
  own clouds), every ancestor (the oracle's systematic resampling of the
  GPU's own outer weights), and sampled new particles (candidate, new x, the
  conditioned and resampled cloud, its propagation and measurement update)
  from their parents' exported state.  A graph-replayed run (each step's
  next look-ahead weights inside the new-cloud launch, as timed) equals the
  step calls bit for bit over the same steps.
* Batched serving workload, 1024 linear-Gaussian filters with N log-uniform
  in [256, 4096] and M in {32, 64, 128}, under the 16-lane tile classes the
  autotuner picks for it: sampled filters of every inner size stepped by the
  oracle from the GPU's exported state, and the run equal to step calls.
"""
import numpy as np
import pytest

import bench
import dpf_synth as S
import paper_1203_2394_amd as dpf
from oracle import ladpf
from oracle import philox as P
from oracle.models import make_model
from oracle.resample import systematic_log, weights_from_log

from parity_util import DELTA, TOL, assert_clean, compare_la, near_tie, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _rows(blob, N, M, dx, dz, rows):
    """x (len, dx), z (len, M, dz) and lam (len, M) of outer particles `rows`
    of a one-filter state blob on the device (only those bytes are copied)."""
    head = 16
    xo = head
    zo = xo + 4 * N * dx
    lo = zo + 4 * N * M * dz
    xs = blob[xo:zo].cpu().numpy().view(np.float32).reshape(dx, N)[:, rows].T.astype(np.float64)
    z = np.stack([blob[zo + 4 * i * M * dz:zo + 4 * (i + 1) * M * dz].cpu().numpy().view(np.float32)
                  .reshape(dz, M).T for i in rows]).astype(np.float64)
    lam = np.stack([blob[lo + 4 * i * M:lo + 4 * (i + 1) * M].cpu().numpy().view(np.float32)
                    for i in rows]).astype(np.float64)
    return xs, z, lam


def test_highdim_full_size_sampled_outputs_match_oracle():
    spec = S.highdim_c4(bench.PARAM_SEED)
    model = make_model(spec.kind, spec.dx, spec.dz, spec.dy, spec.blob)
    N, M, seed = bench.HD_N, bench.HD_M, bench.FILTER_SEED
    dx, dz = spec.dx, spec.dz
    _, _, ys = S.simulate(spec, 3, bench.HD_SEED)
    Y = torch.tensor(ys, dtype=torch.float32, device="cuda").reshape(3, 1, spec.dy).contiguous()
    y1 = Y[0, 0].double().cpu().numpy()

    a = dpf.Filter(spec.kind, dx, dz, spec.dy, spec.blob, [N], [M], seed=seed)
    s0 = a.export_state()
    a.lookahead_step(Y[0])
    ell = a.copy_buffer(dpf.BUF_ELL)
    logw = a.copy_buffer(dpf.BUF_LOGW).cpu().numpy().astype(np.float64)
    anc = a.copy_buffer(dpf.BUF_ANC).cpu().numpy()
    sel = a.copy_buffer(dpf.BUF_SEL).cpu().numpy()
    s1 = a.export_state()
    torch.cuda.synchronize()
    t = 1

    # every ancestor: the oracle's systematic resampling of the GPU's weights
    u_outer = float(P.uniform53(seed, 0, t, 0, P.OUTER_U))
    A_o, deg, _ = systematic_log(logw, N, u_outer)
    assert not deg
    w_out, _, _ = weights_from_log(logw)
    bad = np.nonzero(A_o != anc)[0]
    print("high-dim full size: %d of %d ancestors differ" % (len(bad), N), flush=True)
    assert all(near_tie(w_out, u_outer, N, k, A_o[k], anc[k]) for k in bad)

    # sampled new particles: the most-copied parents' children and a spread
    counts = np.bincount(anc, minlength=N)
    ks = sorted(set([int(np.argmax(anc == int(np.argmax(counts))))] + [0, 1, 777, 4096, 9999, N - 1]))
    parents = sorted(set(int(anc[k]) for k in ks) | {0, 5000, N - 1})
    xp, zp, lamp = _rows(s0, N, M, dx, dz, parents)
    sub = {"x": xp, "z": zp, "lam": lamp, "t": 0}
    xla_o, _, ell_o, logw_o = ladpf.lookahead(model, sub, y1, seed, 0, rows=np.asarray(parents))
    ell_g = np.stack([ell[p * M:(p + 1) * M].cpu().numpy() for p in parents]).astype(np.float64)
    # look-ahead weights of the sampled outer particles, from their own clouds
    e_ell = rel_err(ell_g, ell_o)
    e_logw = rel_err(logw[parents], logw_o)
    print("high-dim full size: err_ell %.3g err_logw %.3g over %d sampled particles"
          % (e_ell, e_logw, len(parents)), flush=True)
    assert e_ell <= TOL and e_logw <= TOL

    xn, zn, lamn = _rows(s1, N, M, dx, dz, ks)
    u_cand = P.uniform53(seed, 0, t, np.arange(N), P.CAND_U)
    u_inner = P.uniform53(seed, 0, t, np.arange(N), P.INNER_U)
    flips = 0
    for q, k in enumerate(ks):
        p = int(anc[k])
        r = parents.index(p)
        # steps 3-4 on the GPU's own weights of the parent (their parity is above)
        xk, zk, lk, c, b, _ = ladpf.new_particle(model, xp[r], zp[r], lamp[r], ell_g[r], xla_o[r], y1, seed, 0,
                                                 t, k, float(u_cand[k]), float(u_inner[k]))
        if c != sel[k]:
            wc, _, _ = weights_from_log(ell_g[r])
            assert near_tie(wc, float(u_cand[k]), 1, 0, c, int(sel[k])), (k, c, sel[k])
            continue
        assert rel_err(xn[q], xk) <= TOL, (k, xn[q], xk)
        # the inner clouds: an ancestor may flip where its point lies at a boundary
        dzr = np.max(np.abs(zn[q] - zk) / np.maximum(1.0, np.abs(zk)), axis=1)
        wk, _, _ = weights_from_log(lamp[r] + model.logpx(xk, xp[r], zp[r], 0))
        C = np.cumsum(wk)
        for j in np.nonzero(dzr > TOL)[0]:
            Pj = ((j + float(u_inner[k])) * C[-1]) / M
            assert abs(Pj - C[b[j]]) <= DELTA * C[-1] or (b[j] > 0 and abs(Pj - C[b[j] - 1]) <= DELTA * C[-1])
            flips += 1
        ok = dzr <= TOL
        assert rel_err(zn[q][ok], zk[ok]) <= TOL
        if ok.all():
            assert rel_err(lamn[q], lk) <= TOL
    print("high-dim full size: %d sampled new particles, %d explained inner flips" % (len(ks), flips), flush=True)
    assert flips <= len(ks) * M // 50

    # the timed form: a graph-replayed run equals the step calls bit for bit
    a.lookahead_step(Y[1])
    s2 = a.export_state()
    ea = a.estimate()
    del s0, s1
    a.close()
    torch.cuda.empty_cache()
    b = dpf.Filter(spec.kind, dx, dz, spec.dy, spec.blob, [N], [M], seed=seed)
    b.run(Y[:2], trace=False, use_graph=True)
    eb = b.estimate()
    assert torch.equal(s2, b.export_state())
    assert torch.equal(ea["xhat"], eb["xhat"]) and torch.equal(ea["loglik"], eb["loglik"])
    torch.cuda.synchronize()
    b.close()


def test_batched_full_size_sampled_filters_match_oracle():
    spec = S.lingauss_c1(False)
    model = make_model(spec.kind, spec.dx, spec.dz, spec.dy, spec.blob)
    rb = S.ragged_batch(F=bench.BATCH_F, seed=bench.BATCH_SEED)
    F, seed = bench.BATCH_F, bench.BATCH_SEED
    classes = dpf.tile_classes()
    cls_of = {32: classes.index((16, 2)), 64: classes.index((16, 4)), 128: classes.index((16, 8))}
    tiling = [cls_of[int(m)] for m in rb.M]
    ys = np.stack([S.simulate(spec, 3, int(rb.data_seeds[f]))[2] for f in range(F)], axis=1)
    Y = torch.tensor(ys, dtype=torch.float32, device="cuda").contiguous()   # [T][F][1]

    a = dpf.Filter(spec.kind, spec.dx, spec.dz, spec.dy, spec.blob, rb.N, rb.M, seed=seed)
    a.set_tiling(tiling)
    st0 = a.unpack_state(a.export_state())
    a.lookahead_step(Y[0])
    out = a.unpack_state(a.export_state())
    ell = a.copy_buffer(dpf.BUF_ELL).cpu().numpy()
    logw = a.copy_buffer(dpf.BUF_LOGW).cpu().numpy()
    anc = a.copy_buffer(dpf.BUF_ANC).cpu().numpy()
    sel = a.copy_buffer(dpf.BUF_SEL).cpu().numpy()
    oo = np.concatenate([[0], np.cumsum(rb.N)]).astype(np.int64)
    io = np.concatenate([[0], np.cumsum(rb.N.astype(np.int64) * rb.M)])
    # two filters of each inner size: the smallest and the largest N
    picks = []
    for m in (32, 64, 128):
        idx = np.nonzero(rb.M == m)[0]
        picks += [int(idx[np.argmin(rb.N[idx])]), int(idx[np.argmax(rb.N[idx])])]
    for f in picks:
        n, m = int(rb.N[f]), int(rb.M[f])
        st32 = {"t": int(st0["t"][f]), "x": st0["x"][f].astype(np.float64), "z": st0["z"][f].astype(np.float64),
                "lam": st0["lam"][f].astype(np.float64)}
        gs = {"x": out["x"][f], "z": out["z"][f], "lam": out["lam"][f]}
        r, _, _ = compare_la(model, st32, ys[0, f].astype(np.float64), seed, f, gs,
                             ell[io[f]:io[f] + n * m].reshape(n, m), logw[oo[f]:oo[f] + n],
                             anc[oo[f]:oo[f] + n], sel[oo[f]:oo[f] + n])
        print("batched full size: filter %d N=%d M=%d class %s: %s" % (f, n, m, classes[tiling[f]], r.line()),
              flush=True)
        assert_clean(r, n=n)

    # the timed form: a graph-replayed run of the tuned handle equals the step calls
    a.lookahead_step(Y[1])
    sa = a.export_state()
    b = dpf.Filter(spec.kind, spec.dx, spec.dz, spec.dy, spec.blob, rb.N, rb.M, seed=seed)
    b.set_tiling(tiling)
    b.run(Y[:2], trace=False, use_graph=True)
    assert torch.equal(sa, b.export_state())
    ea, eb = a.estimate(), b.estimate()
    for k in ("xhat", "zhat", "ess", "loglik"):
        assert torch.equal(ea[k], eb[k]), k
    torch.cuda.synchronize()
