"""Python binding of libdpf.so, the gfx950 look-ahead decentralized particle filter.

Argument marshalling only: every step of the filter runs in the library's HIP
kernels.  PyTorch provides device memory (the caller-owned workspace and the
input / output tensors) and the current HIP stream.  The names mirror
include/dpf.h.  Importing this package does not load the library; the first
call does, and fails loudly if it has not been built
(``python -m paper_1203_2394_amd.build`` or ``__graft_entry__.build()``).
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdpf.so")

DPF_ABI_VERSION = 1
MODEL_LINGAUSS, MODEL_NONLIN, MODEL_HIGHDIM, MODEL_TWODIM, MODEL_FOURDIM, MODEL_TWODIM_ZFIRST = 1, 2, 3, 4, 5, 6
ALGO_LOOKAHEAD, ALGO_PLAIN = 0, 1
FLAG_DEGENERATE_OUTER, FLAG_DEGENERATE_INNER, FLAG_NONFINITE, FLAG_FALLBACK = 1, 2, 4, 8
BUF_ELL, BUF_LOGW, BUF_ANC, BUF_SEL, BUF_MDN, BUF_X, BUF_FALLBACK = range(7)
MLP_BLOB_BYTES = 166272
MLP_NPARAM = 82464
MLP_IN, MLP_HID, MLP_OUT, MLP_MIX = 32, 256, 32, 4

# Every symbol the header declares (checked by the CPU test suite).
EXPORTS = [
    "dpf_workspace_bytes", "dpf_create", "dpf_reset", "dpf_destroy", "dpf_lookahead_step",
    "dpf_step", "dpf_estimate", "dpf_run", "dpf_state_bytes", "dpf_export_state",
    "dpf_import_state", "dpf_copy_buffer", "dpf_last_error", "dpf_philox_words",
    "dpf_normals", "dpf_systematic", "dpf_segmented_systematic", "dpf_set_phase_events",
    "dpf_set_proposal", "dpf_learned_step", "dpf_learned_step_given", "dpf_features",
    "dpf_mlp_blob_bytes", "dpf_mlp_param_count", "dpf_mlp_forward", "dpf_mlp_train_workspace_bytes",
    "dpf_mlp_pack", "dpf_mlp_train_step", "dpf_learned_run", "dpf_tile_classes", "dpf_set_tiling",
    "dpf_estimate_rb", "dpf_systematic_noalloc", "dpf_set_lookahead_companions", "dpf_set_prediction",
    "dpf_predicted_observation", "dpf_feature_stats", "dpf_standardize", "dpf_permutation",
    "dpf_gather_rows",
]


class DPFError(RuntimeError):
    pass


class _Config(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_uint32),
        ("model", ctypes.c_int32),
        ("algo", ctypes.c_int32),
        ("dx", ctypes.c_int32),
        ("dz", ctypes.c_int32),
        ("dy", ctypes.c_int32),
        ("params", ctypes.POINTER(ctypes.c_double)),
        ("n_params", ctypes.c_size_t),
        ("n_filters", ctypes.c_int32),
        ("N", ctypes.POINTER(ctypes.c_int32)),
        ("M", ctypes.POINTER(ctypes.c_int32)),
        ("seed", ctypes.c_uint64),
        ("reserved", ctypes.c_uint32),
    ]


_LIB = None
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_sz = ctypes.c_size_t


def lib():
    """Load libdpf.so (once).  Raises if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise DPFError("libdpf.so is not built at %s; run __graft_entry__.build()" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "dpf_workspace_bytes": (_sz, [ctypes.POINTER(_Config)]),
        "dpf_create": (_i32, [ctypes.POINTER(_Config), _vp, _sz, _vp, ctypes.POINTER(_vp)]),
        "dpf_reset": (_i32, [_vp]),
        "dpf_destroy": (_i32, [_vp]),
        "dpf_lookahead_step": (_i32, [_vp, _vp, _vp]),
        "dpf_step": (_i32, [_vp, _vp, _vp]),
        "dpf_estimate": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp]),
        "dpf_estimate_rb": (_i32, [_vp, _vp]),
        "dpf_run": (_i32, [_vp, _vp, _i32, _vp, _vp, _vp, _i32]),
        "dpf_state_bytes": (_sz, [_vp]),
        "dpf_export_state": (_i32, [_vp, _vp, _sz]),
        "dpf_import_state": (_i32, [_vp, _vp, _sz]),
        "dpf_copy_buffer": (_i32, [_vp, _i32, _vp, _sz]),
        "dpf_last_error": (ctypes.c_char_p, []),
        "dpf_philox_words": (_i32, [ctypes.c_uint64, ctypes.c_uint32, _vp, _sz, _vp, _vp]),
        "dpf_normals": (_i32, [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                               _i32, _i32, _i32, _vp, _vp]),
        "dpf_systematic": (_i32, [_vp, _i32, _i32, ctypes.c_double, _vp, _vp, _vp]),
        "dpf_systematic_noalloc": (_i32, [_vp, _i32, _i32, ctypes.c_double, _vp, _vp]),
        "dpf_segmented_systematic": (_i32, [_vp, _i32, _i32, _i32, _vp, _vp, _vp]),
        "dpf_set_phase_events": (_i32, [_vp, _vp, _i32]),
        "dpf_set_proposal": (_i32, [_vp, _vp, _sz, ctypes.c_double]),
        "dpf_learned_step": (_i32, [_vp, _vp, _vp]),
        "dpf_learned_step_given": (_i32, [_vp, _vp, _vp, _vp, ctypes.c_double]),
        "dpf_features": (_i32, [_vp, _vp, _vp]),
        "dpf_learned_run": (_i32, [_vp, _vp, _i32, _vp, _vp, _vp, _i32]),
        "dpf_tile_classes": (_i32, [_vp, _vp, _i32]),
        "dpf_set_tiling": (_i32, [_vp, _vp]),
        "dpf_set_lookahead_companions": (_i32, [_vp, _i32]),
        "dpf_set_prediction": (_i32, [_vp, _i32, _vp]),
        "dpf_predicted_observation": (_i32, [_vp, _vp]),
        "dpf_mlp_blob_bytes": (_sz, []),
        "dpf_mlp_param_count": (_sz, []),
        "dpf_mlp_forward": (_i32, [_vp, _vp, _i32, _vp, _vp]),
        "dpf_mlp_train_workspace_bytes": (_sz, [_i32]),
        "dpf_mlp_pack": (_i32, [_vp, _vp, _vp, _vp, _vp, _sz, _vp]),
        "dpf_mlp_train_step": (_i32, [_vp, _vp, _vp, _vp, _i32, ctypes.c_float, _i32, _vp, _sz, _vp, _vp,
                                      _vp]),
        "dpf_feature_stats": (_i32, [_vp, ctypes.c_int64, _i32, _i32, _vp, _vp, ctypes.c_float, _vp]),
        "dpf_standardize": (_i32, [_vp, ctypes.c_int64, _i32, _i32, _vp, _vp, _vp, _i32, _vp]),
        "dpf_permutation": (_i32, [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int64, _vp, _vp]),
        "dpf_gather_rows": (_i32, [_vp, ctypes.c_int64, _i32, _i32, _vp, _i32, _vp, _i32, _vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = L
    return L


def _check(status):
    if status != 0:
        msg = lib().dpf_last_error()
        raise DPFError("dpf status %d: %s" % (status, msg.decode() if msg else ""))


def _torch():
    import torch
    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream_ptr(device):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Filter:
    """A batch of F independent filters sharing one model (one library handle).

    ``N`` and ``M`` are per-filter outer and inner particle counts (ints or
    sequences of length F).  ``algo`` is ``"lookahead"`` or ``"plain"``.
    The workspace is a torch uint8 tensor owned by this object.
    """

    def __init__(self, model, dx, dz, dy, params, N, M, seed=0, algo="lookahead", n_filters=None,
                 device="cuda"):
        torch = _torch()
        L = lib()
        if n_filters is None:
            n_filters = len(N) if hasattr(N, "__len__") else 1
        self.F = int(n_filters)
        self.N = np.broadcast_to(np.asarray(N, dtype=np.int32), (self.F,)).copy()
        self.M = np.broadcast_to(np.asarray(M, dtype=np.int32), (self.F,)).copy()
        self.params = np.ascontiguousarray(params, dtype=np.float64)
        self.model, self.dx, self.dz, self.dy = int(model), int(dx), int(dz), int(dy)
        self.algo = {"lookahead": ALGO_LOOKAHEAD, "plain": ALGO_PLAIN}[algo]
        self.device = torch.device(device)
        self.seed = int(seed)
        cfg = _Config()
        cfg.abi_version = DPF_ABI_VERSION
        cfg.model = self.model
        cfg.algo = self.algo
        cfg.dx, cfg.dz, cfg.dy = self.dx, self.dz, self.dy
        cfg.params = self.params.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        cfg.n_params = self.params.size
        cfg.n_filters = self.F
        cfg.N = self.N.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        cfg.M = self.M.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        cfg.seed = self.seed & 0xFFFFFFFFFFFFFFFF
        cfg.reserved = 0
        self._cfg = cfg
        nbytes = L.dpf_workspace_bytes(ctypes.byref(cfg))
        if nbytes == 0:
            _check(1)
        self.workspace_bytes = nbytes
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        self._ws_ptr = (base + 255) & ~255
        h = ctypes.c_void_p()
        _check(L.dpf_create(ctypes.byref(cfg), ctypes.c_void_p(self._ws_ptr), nbytes,
                            _stream_ptr(self.device), ctypes.byref(h)))
        self._h = h
        self.NT = int(self.N.sum())
        self.NMT = int((self.N.astype(np.int64) * self.M).sum())

    # -------------------------------------------------------------- steps
    def _y(self, y):
        torch = _torch()
        y = torch.as_tensor(y, dtype=torch.float32, device=self.device).reshape(self.F, self.dy)
        return y.contiguous()

    def _active(self, active):
        if active is None:
            return None
        torch = _torch()
        return torch.as_tensor(active, dtype=torch.uint8, device=self.device).contiguous()

    def lookahead_step(self, y, active=None):
        y = self._y(y)
        act = self._active(active)
        _check(lib().dpf_lookahead_step(self._h, _ptr(y), _ptr(act)))
        self._keep = (y, act)

    def step(self, y, active=None):
        y = self._y(y)
        act = self._active(active)
        _check(lib().dpf_step(self._h, _ptr(y), _ptr(act)))
        self._keep = (y, act)

    def reset(self):
        _check(lib().dpf_reset(self._h))

    def set_tiling(self, classes):
        """Tile class per filter (index into tile_classes(), or -1 = default)."""
        c = np.ascontiguousarray(np.broadcast_to(np.asarray(classes, dtype=np.int32), (self.F,)))
        _check(lib().dpf_set_tiling(self._h, c.ctypes.data_as(ctypes.c_void_p)))

    def set_prediction(self, enable=True, trace_T=0):
        """Form the predicted observation in every look-ahead step; with
        trace_T > 0 also record it per step in a [trace_T][F] tensor
        (returned; rows indexed by absolute time - 1)."""
        torch = _torch()
        tr = None
        if enable and trace_T > 0:
            tr = torch.full((int(trace_T), self.F), float("nan"), dtype=torch.float32, device=self.device)
        _check(lib().dpf_set_prediction(self._h, int(bool(enable)), _ptr(tr)))
        self._ytrace = tr
        return tr

    def predicted_observation(self):
        torch = _torch()
        out = torch.empty(self.F, dtype=torch.float32, device=self.device)
        _check(lib().dpf_predicted_observation(self._h, _ptr(out)))
        return out

    def set_companions(self, n_comp):
        """Companions per look-ahead candidate: K >= 1 the nested estimator,
        0 the paired form (default)."""
        _check(lib().dpf_set_lookahead_companions(self._h, int(n_comp)))

    # -------------------------------------------------------------- learned proposal
    def set_proposal(self, mlp, ess_frac=0.1):
        """Use the network of ``mlp`` (an MLP) as the outer proposal."""
        _check(lib().dpf_set_proposal(self._h, _ptr(mlp.blob), mlp.blob.numel(), float(ess_frac)))
        self._proposal = mlp

    def learned_step(self, y, active=None):
        y = self._y(y)
        act = self._active(active)
        _check(lib().dpf_learned_step(self._h, _ptr(y), _ptr(act)))
        self._keep = (y, act)

    def learned_step_given(self, y, mdn, ess_frac=0.1, active=None):
        """Learned step with caller-supplied network outputs mdn [sum N][32]."""
        torch = _torch()
        y = self._y(y)
        act = self._active(active)
        mdn = torch.as_tensor(mdn, dtype=torch.float32, device=self.device).reshape(self.NT, MLP_OUT).contiguous()
        _check(lib().dpf_learned_step_given(self._h, _ptr(y), _ptr(act), _ptr(mdn), float(ess_frac)))
        self._keep = (y, act, mdn)

    def features(self, y):
        """Raw features [sum N][32] of the current state for observations y [F][dy]."""
        torch = _torch()
        y = self._y(y)
        out = torch.empty(self.NT, MLP_IN, dtype=torch.float32, device=self.device)
        _check(lib().dpf_features(self._h, _ptr(y), _ptr(out)))
        self._keep = y
        return out

    def estimate(self):
        torch = _torch()
        d = self.device
        out = {
            "xhat": torch.empty(self.F, self.dx, dtype=torch.float32, device=d),
            "zhat": torch.empty(self.F, self.dz, dtype=torch.float32, device=d),
            "ess": torch.empty(self.F, dtype=torch.float32, device=d),
            "loglik": torch.empty(self.F, dtype=torch.float64, device=d),
            "flags": torch.empty(self.F, dtype=torch.int32, device=d),
        }
        _check(lib().dpf_estimate(self._h, _ptr(out["xhat"]), _ptr(out["zhat"]), _ptr(out["ess"]),
                                  _ptr(out["loglik"]), _ptr(out["flags"])))
        return out

    def estimate_rb(self):
        """Rao-Blackwellised x estimate [F][dx] of the look-ahead step just
        taken (dpf_estimate_rb)."""
        torch = _torch()
        out = torch.empty(self.F, self.dx, dtype=torch.float32, device=self.device)
        _check(lib().dpf_estimate_rb(self._h, _ptr(out)))
        return out

    def run(self, Y, Tf=None, trace=True, use_graph=True, learned=False):
        """Run over device-resident observations Y [T][F][dy]; returns traces.
        learned: the learned step (dpf_learned_run) instead of the handle's
        algorithm."""
        torch = _torch()
        Y = torch.as_tensor(Y, dtype=torch.float32, device=self.device).contiguous()
        T = Y.shape[0]
        Tf_t = None if Tf is None else torch.as_tensor(Tf, dtype=torch.int32, device=self.device).contiguous()
        xt = zt = None
        if trace:
            xt = torch.full((T, self.F, self.dx), float("nan"), dtype=torch.float32, device=self.device)
            zt = torch.full((T, self.F, self.dz), float("nan"), dtype=torch.float32, device=self.device)
        fn = lib().dpf_learned_run if learned else lib().dpf_run
        _check(fn(self._h, _ptr(Y), int(T), _ptr(Tf_t), _ptr(xt), _ptr(zt), int(bool(use_graph))))
        self._keep = (Y, Tf_t, xt, zt)
        return xt, zt

    # -------------------------------------------------------------- state
    def state_bytes(self):
        return lib().dpf_state_bytes(self._h)

    def export_state(self):
        torch = _torch()
        buf = torch.empty(self.state_bytes(), dtype=torch.uint8, device=self.device)
        _check(lib().dpf_export_state(self._h, _ptr(buf), buf.numel()))
        return buf

    def import_state(self, buf):
        torch = _torch()
        buf = torch.as_tensor(buf, dtype=torch.uint8, device=self.device).contiguous()
        _check(lib().dpf_import_state(self._h, _ptr(buf), buf.numel()))
        self._keep = buf

    def pack_state(self, t, x, z, lam):
        """Host arrays (per filter lists or single arrays in oracle layout:
        x (N, dx), z (N, M, dz), lam (N, M)) -> uint8 state blob (numpy)."""
        F = self.F
        if F == 1 and not isinstance(x, (list, tuple)):
            t, x, z, lam = [t], [x], [z], [lam]
        tb = (4 * F + 15) & ~15
        head = np.zeros(tb, dtype=np.uint8)
        head[:4 * F] = np.asarray(t, dtype=np.int32).view(np.uint8)
        xs = np.concatenate([np.asarray(xi, dtype=np.float32) for xi in x], axis=0).T.ravel()
        zs = np.concatenate([np.asarray(zi, dtype=np.float32).transpose(0, 2, 1).ravel() for zi in z])
        ls = np.concatenate([np.asarray(li, dtype=np.float32).ravel() for li in lam])
        return np.concatenate([head, xs.view(np.uint8), zs.view(np.uint8), ls.view(np.uint8)])

    def unpack_state(self, blob):
        """uint8 state blob -> dict of per-filter host arrays in oracle layout."""
        b = np.asarray(blob.cpu() if hasattr(blob, "cpu") else blob, dtype=np.uint8)
        F = self.F
        tb = (4 * F + 15) & ~15
        t = b[:4 * F].view(np.int32).copy()
        off = tb
        nx = self.NT * self.dx
        xs = b[off:off + 4 * nx].view(np.float32).reshape(self.dx, self.NT).T
        off += 4 * nx
        nz = self.NMT * self.dz
        zs = b[off:off + 4 * nz].view(np.float32)
        off += 4 * nz
        ls = b[off:off + 4 * self.NMT].view(np.float32)
        out = {"t": t, "x": [], "z": [], "lam": []}
        oo = io = 0
        for f in range(F):
            n, m = int(self.N[f]), int(self.M[f])
            out["x"].append(xs[oo:oo + n].copy())
            out["z"].append(zs[io * self.dz:(io + n * m) * self.dz].reshape(n, self.dz, m).transpose(0, 2, 1).copy())
            out["lam"].append(ls[io:io + n * m].reshape(n, m).copy())
            oo += n
            io += n * m
        return out

    def copy_buffer(self, which):
        torch = _torch()
        sizes = {BUF_ELL: (self.NMT, torch.float32), BUF_LOGW: (self.NT, torch.float32),
                 BUF_ANC: (self.NT, torch.int32), BUF_SEL: (self.NT, torch.int32),
                 BUF_MDN: (self.NT * MLP_OUT, torch.float32), BUF_X: (self.NT * self.dx, torch.float32),
                 BUF_FALLBACK: (self.F, torch.uint8)}
        n, dt = sizes[which]
        out = torch.empty(n, dtype=dt, device=self.device)
        _check(lib().dpf_copy_buffer(self._h, int(which), _ptr(out), out.numel() * out.element_size()))
        return out

    def set_phase_events(self, events):
        """Record torch.cuda.Event objects (created with enable_timing=True) at
        the phase boundaries of the following steps, 5 per step."""
        if not events:
            _check(lib().dpf_set_phase_events(self._h, None, 0))
            self._events = None
            return
        torch = _torch()
        for e in events:
            if not e.cuda_event:  # torch creates the HIP event on first record
                e.record(torch.cuda.current_stream(self.device))
        torch.cuda.synchronize(self.device)
        arr = (ctypes.c_void_p * len(events))(*[ctypes.c_void_p(e.cuda_event) for e in events])
        self._events = (events, arr)
        _check(lib().dpf_set_phase_events(self._h, arr, len(events)))

    def close(self):
        if getattr(self, "_h", None):
            lib().dpf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ primitives
def tile_classes():
    """[(SEG, JPT)] of the built tile classes, by class index."""
    seg = (ctypes.c_int32 * 32)()
    jpt = (ctypes.c_int32 * 32)()
    n = lib().dpf_tile_classes(seg, jpt, 32)
    return [(seg[k], jpt[k]) for k in range(n)]


def philox_words(seed, filter_id, ctr, device="cuda"):
    torch = _torch()
    ctr = torch.as_tensor(np.asarray(ctr, dtype=np.uint32).view(np.int32), device=device).contiguous()
    n = ctr.numel() // 4
    out = torch.empty_like(ctr)
    _check(lib().dpf_philox_words(int(seed) & 0xFFFFFFFFFFFFFFFF, int(filter_id), _ptr(ctr), n, _ptr(out),
                                  _stream_ptr(torch.device(device))))
    return out.cpu().numpy().view(np.uint32).reshape(n, 4)


def normals(seed, filter_id, t, purpose, n_a, n_b, D, device="cuda"):
    torch = _torch()
    out = torch.empty(n_a * n_b * D, dtype=torch.float32, device=device)
    _check(lib().dpf_normals(int(seed) & 0xFFFFFFFFFFFFFFFF, int(filter_id), int(t), int(purpose), int(n_a),
                             int(n_b), int(D), _ptr(out), _stream_ptr(torch.device(device))))
    return out.reshape(n_a, n_b, D)


def systematic(w, n_out, u, device="cuda"):
    torch = _torch()
    w = torch.as_tensor(w, dtype=torch.float64, device=device).contiguous()
    scratch = torch.empty(4 * ((w.numel() + 255) // 256), dtype=torch.float64, device=device)
    out = torch.empty(int(n_out), dtype=torch.int32, device=device)
    _check(lib().dpf_systematic(_ptr(w), w.numel(), int(n_out), float(u), _ptr(scratch), _ptr(out),
                                _stream_ptr(torch.device(device))))
    return out


def segmented_systematic(w, n_out, u, device="cuda"):
    torch = _torch()
    w = torch.as_tensor(w, dtype=torch.float64, device=device).contiguous()
    S, n = w.shape
    u = torch.as_tensor(u, dtype=torch.float64, device=device).contiguous()
    out = torch.empty(S, int(n_out), dtype=torch.int32, device=device)
    _check(lib().dpf_segmented_systematic(_ptr(w), int(S), int(n), int(n_out), _ptr(u), _ptr(out),
                                          _stream_ptr(torch.device(device))))
    return out


# ------------------------------------------------------------------ network
_PARAM_SHAPES = [("W1", (MLP_HID, MLP_IN)), ("b1", (MLP_HID,)), ("W2", (MLP_HID, MLP_HID)),
                 ("b2", (MLP_HID,)), ("W3", (MLP_OUT, MLP_HID)), ("b3", (MLP_OUT,))]


def flatten_params(p):
    """Dict of arrays (W3 / b3 may have fewer than 32 output rows) -> FP32
    parameter vector in the library's order, zero-padded."""
    out = np.zeros(MLP_NPARAM, dtype=np.float32)
    off = 0
    for name, shape in _PARAM_SHAPES:
        a = np.zeros(shape, dtype=np.float64)
        v = np.asarray(p[name], dtype=np.float64)
        a[tuple(slice(0, k) for k in v.shape)] = v
        n = int(np.prod(shape))
        out[off:off + n] = a.ravel()
        off += n
    return out


def unflatten_params(v):
    v = np.asarray(v, dtype=np.float64)
    out, off = {}, 0
    for name, shape in _PARAM_SHAPES:
        n = int(np.prod(shape))
        out[name] = v[off:off + n].reshape(shape).copy()
        off += n
    return out


def init_params(seed, n_feat, n_used_out=20):
    """He-style initial parameters (zero biases, zero padding columns / rows)."""
    g = np.random.Generator(np.random.PCG64(seed))
    p = {name: np.zeros(shape) for name, shape in _PARAM_SHAPES}
    p["W1"][:, :n_feat] = g.normal(0.0, np.sqrt(2.0 / n_feat), size=(MLP_HID, n_feat))
    p["W2"] = g.normal(0.0, np.sqrt(2.0 / MLP_HID), size=(MLP_HID, MLP_HID))
    p["W3"][:n_used_out] = g.normal(0.0, 0.1 * np.sqrt(1.0 / MLP_HID), size=(n_used_out, MLP_HID))
    return p


class MLP:
    """The proposal network on the device: FP32 parameters with Adam moments
    (``state`` [3][NPARAM]), the BF16 blob the filters and the forward kernel
    read, and a training workspace for batch ``batch``."""

    def __init__(self, params, fmean, fstd, batch=4096, device="cuda"):
        torch = _torch()
        self.device = torch.device(device)
        vec = params if isinstance(params, np.ndarray) and params.ndim == 1 else flatten_params(params)
        self.state = torch.zeros(3, MLP_NPARAM, dtype=torch.float32, device=self.device)
        self.state[0] = torch.as_tensor(np.asarray(vec, dtype=np.float32), device=self.device)
        fm = np.zeros(MLP_IN, dtype=np.float32)
        fs = np.ones(MLP_IN, dtype=np.float32)
        fm[:len(fmean)] = fmean
        fs[:len(fstd)] = fstd
        self.fmean = torch.as_tensor(fm, device=self.device)
        self.fstd = torch.as_tensor(fs, device=self.device)
        self.blob = torch.zeros(MLP_BLOB_BYTES, dtype=torch.uint8, device=self.device)
        self.batch = int(batch)
        nb = lib().dpf_mlp_train_workspace_bytes(self.batch)
        if nb == 0:
            raise DPFError("batch %d must be a positive multiple of 32" % self.batch)
        self._ws = torch.empty(nb, dtype=torch.uint8, device=self.device)
        self.adam_t = 0
        self.pack()

    def _stream(self):
        return _stream_ptr(self.device)

    def pack(self):
        """Blob (and the training copies) from the current FP32 parameters."""
        _check(lib().dpf_mlp_pack(_ptr(self.state[0]), _ptr(self.fmean), _ptr(self.fstd), _ptr(self.blob),
                                  _ptr(self._ws), self._ws.numel(), self._stream()))

    def params(self):
        return unflatten_params(self.state[0].cpu().numpy())

    def forward(self, X):
        """Standardised features X [B][32] -> outputs [B][32]."""
        torch = _torch()
        X = torch.as_tensor(X, dtype=torch.float32, device=self.device).contiguous()
        out = torch.empty(X.shape[0], MLP_OUT, dtype=torch.float32, device=self.device)
        _check(lib().dpf_mlp_forward(_ptr(self.blob), _ptr(X), int(X.shape[0]), _ptr(out), self._stream()))
        self._keep = X
        return out

    def _step(self, X, xt, lr, adam_t, want_grad, loss=None):
        torch = _torch()
        X = torch.as_tensor(X, dtype=torch.float32, device=self.device).contiguous()
        xt = torch.as_tensor(xt, dtype=torch.float32, device=self.device).contiguous()
        if X.shape[0] != self.batch:
            raise DPFError("batch of %d rows, network built for %d" % (X.shape[0], self.batch))
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device=self.device)
        grad = torch.empty(MLP_NPARAM, dtype=torch.float32, device=self.device) if want_grad else None
        _check(lib().dpf_mlp_train_step(_ptr(self.state), _ptr(self.blob), _ptr(X), _ptr(xt), self.batch,
                                        float(lr), int(adam_t), _ptr(self._ws), self._ws.numel(), _ptr(loss),
                                        _ptr(grad), self._stream()))
        self._keep = (X, xt)
        return loss, grad

    def train_step(self, X, xt, lr=1e-3, want_grad=False, loss=None):
        """One Adam step on a batch (standardised features, targets [B][2]);
        loss: an optional one-element device tensor (view) for the batch's
        mean NLL."""
        self.adam_t += 1
        return self._step(X, xt, lr, self.adam_t, want_grad, loss)

    def loss_and_grad(self, X, xt):
        """Mean NLL and its gradient at the current parameters (no update)."""
        return self._step(X, xt, 0.0, 0, True)
