"""Training-set preparation on the device (dpf_feature_stats,
dpf_standardize, dpf_permutation, dpf_gather_rows) against NumPy."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1203_2394_amd as dpf  # noqa: E402


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _s():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(st):
    assert st == 0, dpf.lib().dpf_last_error()


@pytest.mark.parametrize("n,cols,ld", [(2, 1, 1), (5000, 26, 26), (40001, 26, 32), (300, 40, 45)])
def test_feature_stats_match_numpy(n, cols, ld):
    g = np.random.default_rng(n)
    X = (g.normal(size=(n, ld)) * g.uniform(0.1, 5, size=ld) + g.normal(size=ld) * 3).astype(np.float32)
    if cols > 3:
        X[:, 3] = 2.5  # a constant column: standard deviation floored
    d = torch.from_numpy(X).cuda()
    m = torch.empty(cols, device="cuda")
    s = torch.empty(cols, device="cuda")
    _check(dpf.lib().dpf_feature_stats(_p(d), n, cols, ld, _p(m), _p(s), ctypes.c_float(1e-3), _s()))
    X64 = X[:, :cols].astype(np.float64)
    mref = X64.mean(axis=0)
    sref = np.maximum(X64.std(axis=0, ddof=1), 1e-3)
    assert np.allclose(m.cpu().numpy(), mref, rtol=1e-6, atol=1e-6)
    assert np.allclose(s.cpu().numpy(), sref, rtol=1e-6, atol=1e-7)
    if cols > 3:
        assert float(s[3]) == np.float32(1e-3)
    # fixed order: the same bits twice
    m2 = torch.empty_like(m)
    s2 = torch.empty_like(s)
    _check(dpf.lib().dpf_feature_stats(_p(d), n, cols, ld, _p(m2), _p(s2), ctypes.c_float(1e-3), _s()))
    assert torch.equal(m, m2) and torch.equal(s, s2)


def test_standardize_is_the_fp32_formula_and_pads_with_zeros():
    g = np.random.default_rng(3)
    n, cols, ld, ld_out = 777, 26, 26, 32
    X = g.normal(size=(n, ld)).astype(np.float32) * 4 + 1
    mean = g.normal(size=cols).astype(np.float32)
    std = g.uniform(0.5, 3, size=cols).astype(np.float32)
    out = torch.full((n, ld_out), 7.0, device="cuda")
    dX, dm, ds = (torch.from_numpy(v).cuda() for v in (X, mean, std))  # held until the kernel has run
    _check(dpf.lib().dpf_standardize(_p(dX), n, cols, ld, _p(dm), _p(ds), _p(out), ld_out, _s()))
    torch.cuda.synchronize()
    ref = np.zeros((n, ld_out), dtype=np.float32)
    ref[:, :cols] = (X[:, :cols] - mean) / std
    assert np.array_equal(out.cpu().numpy(), ref)


@pytest.mark.parametrize("n", [1, 2, 3, 17, 1000, 4096 * 3 + 7, 1 << 20, 1000003])
def test_permutation_is_a_permutation_and_keyed(n):
    p = torch.empty(n, dtype=torch.int32, device="cuda")
    _check(dpf.lib().dpf_permutation(5, 0, n, _p(p), _s()))
    a = p.cpu().numpy()
    assert np.array_equal(np.sort(a), np.arange(n))
    q = torch.empty_like(p)
    _check(dpf.lib().dpf_permutation(5, 0, n, _p(q), _s()))
    assert torch.equal(p, q)
    if n >= 17:
        _check(dpf.lib().dpf_permutation(5, 1, n, _p(q), _s()))
        b = q.cpu().numpy()
        assert np.array_equal(np.sort(b), np.arange(n))
        assert np.mean(a == b) < 0.2
        _check(dpf.lib().dpf_permutation(6, 0, n, _p(q), _s()))
        assert np.mean(a == q.cpu().numpy()) < 0.2
    if n >= 1000:
        # a shuffle, not a near-identity: positions move far on average and
        # the first tenth of the output draws evenly from the input
        assert np.mean(np.abs(a - np.arange(n))) > n / 5
        head = a[: n // 10]
        frac_low = np.mean(head < n // 2)
        assert abs(frac_low - 0.5) < 0.1


def test_gather_rows_bit_exact_and_nan_outside():
    g = np.random.default_rng(9)
    n, cols, ld = 1000, 30, 32
    src = g.normal(size=(n, ld)).astype(np.float32)
    idx = g.integers(0, n, size=333).astype(np.int32)
    idx[5] = n  # outside: a NaN row
    idx[6] = -1
    dst = torch.zeros(333, 34, device="cuda")
    dsrc, didx = torch.from_numpy(src).cuda(), torch.from_numpy(idx).cuda()  # held until the kernel has run
    _check(dpf.lib().dpf_gather_rows(_p(dsrc), n, cols, ld, _p(didx), 333, _p(dst), 34, _s()))
    torch.cuda.synchronize()
    d = dst.cpu().numpy()
    ok = (idx >= 0) & (idx < n)
    assert np.array_equal(d[ok, :cols], src[idx[ok], :cols])
    assert np.all(np.isnan(d[~ok, :cols]))
    assert np.all(d[:, cols:] == 0)
