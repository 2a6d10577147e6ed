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
MODEL_LINGAUSS, MODEL_NONLIN, MODEL_HIGHDIM = 1, 2, 3
ALGO_LOOKAHEAD, ALGO_PLAIN = 0, 1
FLAG_DEGENERATE_OUTER, FLAG_DEGENERATE_INNER, FLAG_NONFINITE, FLAG_FALLBACK = 1, 2, 4, 8
BUF_ELL, BUF_LOGW, BUF_ANC, BUF_SEL = range(4)

# Every symbol the header declares (checked by the CPU test suite).
EXPORTS = [
    "dpf_workspace_bytes", "dpf_create", "dpf_reset", "dpf_destroy", "dpf_lookahead_step",
    "dpf_step", "dpf_estimate", "dpf_run", "dpf_state_bytes", "dpf_export_state",
    "dpf_import_state", "dpf_copy_buffer", "dpf_last_error", "dpf_philox_words",
    "dpf_normals", "dpf_systematic", "dpf_segmented_systematic", "dpf_set_phase_events",
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
        "dpf_segmented_systematic": (_i32, [_vp, _i32, _i32, _i32, _vp, _vp, _vp]),
        "dpf_set_phase_events": (_i32, [_vp, _vp, _i32]),
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

    def run(self, Y, Tf=None, trace=True, use_graph=True):
        """Run over device-resident observations Y [T][F][dy]; returns traces."""
        torch = _torch()
        Y = torch.as_tensor(Y, dtype=torch.float32, device=self.device).contiguous()
        T = Y.shape[0]
        Tf_t = None if Tf is None else torch.as_tensor(Tf, dtype=torch.int32, device=self.device).contiguous()
        xt = zt = None
        if trace:
            xt = torch.full((T, self.F, self.dx), float("nan"), dtype=torch.float32, device=self.device)
            zt = torch.full((T, self.F, self.dz), float("nan"), dtype=torch.float32, device=self.device)
        _check(lib().dpf_run(self._h, _ptr(Y), int(T), _ptr(Tf_t), _ptr(xt), _ptr(zt), int(bool(use_graph))))
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
                 BUF_ANC: (self.NT, torch.int32), BUF_SEL: (self.NT, torch.int32)}
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
