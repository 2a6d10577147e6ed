"""The C interface: the library loads on a machine without a GPU, exports every
symbol include/dpf.h declares, and its host-side validation works (no
compute calls here)."""
import ctypes
import os
import re

import numpy as np
import pytest

import dpf_synth as S
import paper_1203_2394_amd as dpf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dpf.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dpf_[a-z_]+)\s*\(", txt)))


def _lib():
    if not os.path.exists(dpf.LIB_PATH):
        pytest.skip("libdpf.so not built")
    return dpf.lib()


def test_header_and_binding_agree():
    assert _declared() == sorted(dpf.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = _lib()
    for name in _declared():
        assert hasattr(L, name), name


def _cfg(spec, N, M, algo=0, n_params=None):
    c = dpf._Config()
    c.abi_version = 1
    c.model, c.algo = spec.kind, algo
    c.dx, c.dz, c.dy = spec.dx, spec.dz, spec.dy
    blob = np.ascontiguousarray(spec.blob)
    c.params = blob.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    c.n_params = blob.size if n_params is None else n_params
    Na = np.asarray(N, dtype=np.int32)
    Ma = np.asarray(M, dtype=np.int32)
    c.n_filters = len(Na)
    c.N = Na.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    c.M = Ma.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    c.seed = 1
    return c, (blob, Na, Ma)


def test_workspace_bytes_scales_with_sizes():
    L = _lib()
    spec = S.nonlin_c2()
    c1, keep1 = _cfg(spec, [4096], [256])
    c2, keep2 = _cfg(spec, [4096, 100], [256, 50])
    b1 = L.dpf_workspace_bytes(ctypes.byref(c1))
    b2 = L.dpf_workspace_bytes(ctypes.byref(c2))
    # two copies of z (8 floats) and lam, plus ell: at least 76 bytes per inner particle
    assert b1 >= 4096 * 256 * (2 * 8 * 4 + 3 * 4)
    assert b2 > b1


def test_validation_errors_are_reported():
    L = _lib()
    spec = S.nonlin_c2()
    bad = [
        _cfg(spec, [4096], [256], n_params=3),        # wrong parameter count
        _cfg(spec, [4096], [5000]),                   # M too large
        _cfg(spec, [0], [16]),                        # N = 0
        _cfg(spec, [16], [16], algo=7),               # unknown algo
    ]
    for c, keep in bad:
        assert L.dpf_workspace_bytes(ctypes.byref(c)) == 0
        assert len(L.dpf_last_error()) > 0
    c, keep = _cfg(S.ModelSpec(2, 3, 8, 8, spec.blob), [16], [16])
    assert L.dpf_workspace_bytes(ctypes.byref(c)) == 0
    assert b"not built" in L.dpf_last_error()


def test_create_rejects_small_or_misaligned_workspace():
    L = _lib()
    spec = S.lingauss_c1()
    c, keep = _cfg(spec, [100], [50])
    need = L.dpf_workspace_bytes(ctypes.byref(c))
    h = ctypes.c_void_p()
    # host-side checks fail before any device work is queued
    assert L.dpf_create(ctypes.byref(c), ctypes.c_void_p(256), need - 1, None, ctypes.byref(h)) == 2
    assert L.dpf_create(ctypes.byref(c), ctypes.c_void_p(257), need, None, ctypes.byref(h)) == 1
    assert L.dpf_create(ctypes.byref(c), None, need, None, ctypes.byref(h)) == 1


def test_network_sizes_and_batch_validation():
    L = _lib()
    L.dpf_mlp_blob_bytes.restype = ctypes.c_size_t
    L.dpf_mlp_param_count.restype = ctypes.c_size_t
    L.dpf_mlp_train_workspace_bytes.restype = ctypes.c_size_t
    L.dpf_mlp_train_workspace_bytes.argtypes = [ctypes.c_int32]
    hdr = open(os.path.join(ROOT, "include", "dpf.h")).read()
    blob = int(re.search(r"DPF_MLP_BLOB_BYTES\s+(\d+)u", hdr).group(1))
    npar = int(re.search(r"DPF_MLP_NPARAM\s+(\d+)u", hdr).group(1))
    assert L.dpf_mlp_blob_bytes() == blob == dpf.MLP_BLOB_BYTES
    assert L.dpf_mlp_param_count() == npar == dpf.MLP_NPARAM
    # 256x32 + 256 + 256x256 + 256 + 32x256 + 32 parameters
    assert npar == 256 * 32 + 256 + 256 * 256 + 256 + 32 * 256 + 32
    for bad in (0, 16, 31, 33, 4100, (1 << 20) + 32):
        assert L.dpf_mlp_train_workspace_bytes(bad) == 0
    assert L.dpf_mlp_train_workspace_bytes(4096) > 4096 * 256 * 4 * 2


def test_learned_calls_reject_null_handles():
    L = _lib()
    assert L.dpf_learned_step(None, None, None) == 1
    assert L.dpf_set_proposal(None, None, ctypes.c_size_t(0), ctypes.c_double(0.1)) == 1
    assert L.dpf_features(None, None, None) == 1
    L.dpf_mlp_forward.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                  ctypes.c_void_p]
    assert L.dpf_mlp_forward(None, None, 4, None, None) == 1


def test_tile_class_table():
    classes = dpf.tile_classes()
    assert classes[:6] == [(32, 1), (64, 1), (128, 1), (64, 4), (256, 4), (256, 16)]
    assert set(classes[6:]) == {(32, 2), (32, 4), (64, 2), (256, 1), (128, 2), (16, 2), (16, 4), (16, 8)}
    assert all(256 % seg == 0 for seg, _ in classes)
    assert _lib().dpf_set_tiling(None, None) == 1


def test_table1_models_are_built_and_their_noise_covariances_checked():
    L = _lib()
    for spec in (S.twodim_table1(), S.fourdim_table1()):
        c, keep = _cfg(spec, [100], [20])
        assert L.dpf_workspace_bytes(ctypes.byref(c)) > 0, L.dpf_last_error()
    # a cross covariance as large as the variances is not positive definite
    c, keep = _cfg(S.twodim_table1(qx=1.0, qz=1.0, cxz=1.0), [100], [20])
    assert L.dpf_workspace_bytes(ctypes.byref(c)) == 0
    assert b"positive definite" in L.dpf_last_error()
    spec = S.fourdim_table1()
    blob = spec.blob.copy()
    blob[8] = 4.0                                     # cz^2 > qz1 qz2 = 10
    c, keep = _cfg(S.ModelSpec(spec.kind, 2, 2, 1, blob), [100], [20])
    assert L.dpf_workspace_bytes(ctypes.byref(c)) == 0
    assert b"positive definite" in L.dpf_last_error()


def test_model_ids_agree_across_header_binding_and_inputs():
    txt = open(HEADER).read()
    ids = {k: int(v) for k, v in re.findall(r"DPF_MODEL_([A-Z_]+)\s*=\s*(\d+)", txt)}
    assert ids == {"LINGAUSS": 1, "NONLIN": 2, "HIGHDIM": 3, "TWODIM": 4, "FOURDIM": 5, "TWODIM_ZFIRST": 6}
    for name, v in ids.items():
        assert getattr(dpf, "MODEL_" + name) == v
        assert getattr(S, name) == v


def test_training_set_calls_validate_on_the_host():
    """The training-set calls reject bad sizes and null buffers before any
    launch (no device needed); empty requests succeed."""
    L = _lib()
    c_f = ctypes.c_float
    EINVAL = 1
    buf = ctypes.c_void_p(16)  # never dereferenced: the arguments are rejected first
    assert L.dpf_feature_stats(None, 100, 3, 3, None, None, c_f(1e-3), None) == EINVAL
    assert L.dpf_feature_stats(buf, 1, 3, 3, buf, buf, c_f(1e-3), None) == EINVAL       # n < 2
    assert L.dpf_feature_stats(buf, 10, 4, 3, buf, buf, c_f(1e-3), None) == EINVAL      # cols > ld
    assert L.dpf_feature_stats(buf, 10, 3, 3, buf, buf, c_f(-1.0), None) == EINVAL      # negative floor
    assert L.dpf_standardize(buf, 10, 5, 4, buf, buf, buf, 8, None) == EINVAL           # cols > ld
    assert L.dpf_standardize(buf, 0, 3, 3, buf, buf, buf, 8, None) == 0                 # nothing to do
    assert L.dpf_permutation(1, 0, -1, buf, None) == EINVAL
    assert L.dpf_permutation(1, 0, 1 << 31, buf, None) == EINVAL
    assert L.dpf_permutation(1, 0, 0, None, None) == 0
    assert L.dpf_permutation(1, 0, 5, None, None) == EINVAL
    assert L.dpf_gather_rows(buf, 10, 3, 2, buf, 4, buf, 3, None) == EINVAL             # cols > ld_src
    assert L.dpf_gather_rows(None, 10, 3, 3, None, 0, None, 3, None) == 0               # count 0


def test_run_calls_reject_null_handles():
    # both runs check their handle before touching it
    L = _lib()
    for fn in (L.dpf_run, L.dpf_learned_run):
        assert fn(None, ctypes.c_void_p(256), 4, None, None, None, 1) == 1
        assert len(L.dpf_last_error()) > 0
        assert fn(None, None, 4, None, None, None, 0) == 1


def test_normals_call_validates_on_the_host():
    """dpf_normals serves the built draw lengths only (the packed layout's
    ten per two blocks included) and rejects the rest before any launch."""
    L = _lib()
    EINVAL, EUNSUPPORTED = 1, 5
    buf = ctypes.c_void_p(16)  # never dereferenced: rejected or empty first
    assert L.dpf_normals(1, 0, 1, 3, 4, 4, 3, buf, None) == EUNSUPPORTED
    assert "built: 1, 2, 4, 8, 10, 64, 68" in L.dpf_last_error().decode()
    assert L.dpf_normals(1, 0, 1, 3, -1, 4, 10, buf, None) == EINVAL
    assert L.dpf_normals(1, 0, 1, 3, 4, 4, 10, None, None) == EINVAL
    for D in (1, 2, 4, 8, 10, 64, 68):
        assert L.dpf_normals(1, 0, 1, 3, 0, 4, D, buf, None) == 0  # nothing to draw
