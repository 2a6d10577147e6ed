"""dpf_systematic_noalloc (no scratch argument, library-owned device array)
against dpf_systematic (caller's scratch) through the C interface: the same
ancestors bit for bit, on two calls in a row, the second with a smaller
input (the array keeps the first call's group statistics, which the second
must not read)."""
import ctypes

import numpy as np
import pytest

import paper_1203_2394_amd as dpf

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _weights(n, seed):
    g = np.random.default_rng(seed)
    w = np.exp(g.normal(size=n) * 3.0)
    w[g.random(n) < 0.2] = 0.0           # some zero weights
    w[0] = max(w[0], 1e-3)
    return torch.tensor(w, dtype=torch.float64, device="cuda")


def _with_scratch(L, w, n_out, u, stream):
    n = w.numel()
    scratch = torch.empty(4 * ((n + 255) // 256), dtype=torch.float64, device="cuda")
    out = torch.empty(n_out, dtype=torch.int32, device="cuda")
    assert L.dpf_systematic(ctypes.c_void_p(w.data_ptr()), n, n_out, u, ctypes.c_void_p(scratch.data_ptr()),
                            ctypes.c_void_p(out.data_ptr()), stream) == 0, L.dpf_last_error()
    return out


def _no_alloc(L, w, n_out, u, stream):
    out = torch.empty(n_out, dtype=torch.int32, device="cuda")
    assert L.dpf_systematic_noalloc(ctypes.c_void_p(w.data_ptr()), w.numel(), n_out, u,
                                    ctypes.c_void_p(out.data_ptr()), stream) == 0, L.dpf_last_error()
    return out


def test_no_alloc_systematic_equals_the_scratch_version():
    L = dpf.lib()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    cases = [(65536, 65536, 0.37, 1), (3000, 4100, 0.91, 2), (257, 9, 0.05, 3), (1, 5, 0.5, 4)]
    for n, n_out, u, seed in cases:
        w = _weights(n, seed)
        print("no-alloc systematic n=%d n_out=%d" % (n, n_out), flush=True)
        a = _no_alloc(L, w, n_out, u, stream)
        b = _with_scratch(L, w, n_out, u, stream)
        torch.cuda.synchronize()
        assert torch.equal(a, b), (n, n_out)
        c = a.cpu().numpy()
        assert np.all(np.diff(c) >= 0) and c.min() >= 0 and c.max() < n
        assert np.all(w.cpu().numpy()[c] > 0)


def test_no_alloc_rejects_sizes_beyond_its_array():
    L = dpf.lib()
    assert L.dpf_systematic_noalloc(ctypes.c_void_p(256), 65537, 4, 0.5, ctypes.c_void_p(256), None) == 5
    assert b"65536" in L.dpf_last_error()
    assert L.dpf_systematic_noalloc(None, 16, 4, 0.5, None, None) == 1
