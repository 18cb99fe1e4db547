"""Python binding of libdinr (include/dinr.h).

Argument marshalling only: every step of the forward projection, the adjoint
and the training step runs in the library's gfx950 kernels.  torch supplies
device memory and the current stream.  There is no fallback: if libdinr.so is
missing or cannot be loaded, every entry point raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdinr.so")

OK, EINVAL, ENOMEM, EHIP, ENONFINITE, EBUSY, EIO = 0, -1, -2, -3, -4, -5, -6
FP32, BF16 = 0, 1
_NAMES = {EINVAL: "DINR_EINVAL", ENOMEM: "DINR_ENOMEM", EHIP: "DINR_EHIP",
          ENONFINITE: "DINR_ENONFINITE", EBUSY: "DINR_EBUSY", EIO: "DINR_EIO"}


class DinrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class Geometry(C.Structure):
    _fields_ = [("kind", C.c_int32), ("rows", C.c_int32), ("cols", C.c_int32),
                ("n_views", C.c_int32), ("fov_kind", C.c_int32), ("reserved", C.c_int32),
                ("sod", C.c_double), ("sdd", C.c_double), ("pitch_u", C.c_double),
                ("pitch_v", C.c_double), ("off_u", C.c_double), ("off_v", C.c_double),
                ("fov", C.c_double * 6), ("t0", C.c_double), ("t1", C.c_double),
                ("theta", C.POINTER(C.c_double)), ("time", C.POINTER(C.c_double))]


class MLP(C.Structure):
    _fields_ = [("n_freq", C.c_int32), ("width", C.c_int32), ("depth", C.c_int32),
                ("act", C.c_int32), ("out_act", C.c_int32), ("precision", C.c_int32),
                ("recompute", C.c_int32), ("reserved", C.c_int32), ("mu0", C.c_double)]


class Sampling(C.Structure):
    _fields_ = [("mode", C.c_int32), ("n", C.c_int32), ("n_min", C.c_int32),
                ("n_max", C.c_int32), ("h", C.c_double), ("sub", C.c_int32),
                ("jitter", C.c_int32), ("seed", C.c_uint32), ("reserved", C.c_uint32)]


class Request(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n", C.c_int32), ("z_or_theta", C.c_double),
                ("t", C.c_double), ("samples_per_ray", C.c_int32), ("reserved", C.c_int32)]


class Adam(C.Structure):
    _fields_ = [("m_d", C.c_void_p), ("v_d", C.c_void_p), ("lr", C.c_float),
                ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("step", C.c_int64)]


EXPORTS = ["dinr_create", "dinr_destroy", "dinr_last_error", "dinr_num_params",
           "dinr_forward_project", "dinr_project_backward", "dinr_step", "dinr_step_status",
           "dinr_profile_enable", "dinr_profile_read", "dinr_server_create", "dinr_server_destroy",
           "dinr_query", "dinr_poll", "dinr_query_wait", "dinr_query_release",
           "dinr_server_stats", "dinr_probe_mfma", "dinr_set_sample_epoch", "dinr_volume_write",
           "dinr_forward_project_noalloc"]
QUERY_SLICE, QUERY_REPROJECTION = 0, 1


class Volume(C.Structure):
    _fields_ = [("n", C.c_int32), ("nz", C.c_int32), ("nt", C.c_int32), ("slots", C.c_int32),
                ("times", C.POINTER(C.c_double))]


class VolumeStats(C.Structure):
    _fields_ = [("bytes", C.c_int64), ("seconds", C.c_double), ("voxels_per_s", C.c_double)]
PROF_MLP_FWD, PROF_MLP_BWD, PROF_WGRAD, PROF_MLP_FUSED = 0, 1, 2, 3
PROF_RAYS, PROF_LOSS, PROF_REDUCE = 4, 5, 6

_lib = None


def load(path: str = LIB_PATH):
    """Load libdinr.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libdinr.so not built ({path}); run __graft_entry__.build()")
    L = C.CDLL(path)
    vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int
    L.dinr_create.argtypes = [C.POINTER(Geometry), C.POINTER(MLP), C.POINTER(Sampling),
                              C.POINTER(C.c_float), C.c_size_t, C.POINTER(vp)]
    L.dinr_create.restype = i32
    L.dinr_destroy.argtypes = [vp]
    L.dinr_destroy.restype = i32
    L.dinr_last_error.argtypes = [vp]
    L.dinr_last_error.restype = C.c_char_p
    L.dinr_set_sample_epoch.argtypes = [vp, C.c_uint32]
    L.dinr_set_sample_epoch.restype = C.c_int
    L.dinr_num_params.argtypes = [vp]
    L.dinr_num_params.restype = i64
    L.dinr_forward_project.argtypes = [vp, vp, vp, i64, vp, vp, vp]
    L.dinr_forward_project.restype = i32
    L.dinr_forward_project_noalloc.argtypes = [vp, vp, vp, i64, vp, vp, vp]
    L.dinr_forward_project_noalloc.restype = i32
    L.dinr_project_backward.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp]
    L.dinr_project_backward.restype = i32
    L.dinr_step.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp, vp, C.POINTER(Adam), vp]
    L.dinr_step.restype = i32
    L.dinr_step_status.argtypes = [vp, vp]
    L.dinr_step_status.restype = i32
    L.dinr_profile_enable.argtypes = [vp, i32]
    L.dinr_profile_enable.restype = i32
    L.dinr_profile_read.argtypes = [vp, i32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    L.dinr_profile_read.restype = i32
    L.dinr_probe_mfma.argtypes = [i32, i64, vp, C.POINTER(C.c_double)]
    L.dinr_probe_mfma.restype = i32
    L.dinr_server_create.argtypes = [vp, vp, C.c_size_t, C.c_int32, C.POINTER(vp)]
    L.dinr_server_create.restype = i32
    L.dinr_server_destroy.argtypes = [vp]
    L.dinr_server_destroy.restype = i32
    L.dinr_query.argtypes = [vp, C.POINTER(Request), vp, C.POINTER(C.c_uint64)]
    L.dinr_query.restype = i32
    L.dinr_poll.argtypes = [vp, C.c_uint64, C.POINTER(C.c_int32), C.POINTER(C.c_double)]
    L.dinr_poll.restype = i32
    L.dinr_query_wait.argtypes = [vp, C.c_uint64]
    L.dinr_query_wait.restype = i32
    L.dinr_query_release.argtypes = [vp, C.c_uint64]
    L.dinr_query_release.restype = i32
    L.dinr_server_stats.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                    C.POINTER(C.c_size_t), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_int32)]
    L.dinr_server_stats.restype = i32
    L.dinr_volume_write.argtypes = [vp, C.POINTER(Volume), C.c_char_p, C.POINTER(VolumeStats)]
    L.dinr_volume_write.restype = i32
    _lib = L
    return L


def _geometry(g, keep: list) -> Geometry:
    th = np.ascontiguousarray(np.asarray(g.theta, dtype=np.float64))
    tt = np.ascontiguousarray(np.asarray(g.time, dtype=np.float64))
    keep += [th, tt]
    s = Geometry()
    s.kind, s.rows, s.cols, s.n_views, s.fov_kind = g.kind, g.rows, g.cols, g.n_views, g.fov_kind
    s.sod, s.sdd, s.pitch_u, s.pitch_v, s.off_u, s.off_v = (g.sod, g.sdd, g.pitch_u, g.pitch_v,
                                                           g.off_u, g.off_v)
    for k in range(6):
        s.fov[k] = g.fov[k] if k < len(g.fov) else 0.0
    s.t0, s.t1 = g.t0, g.t1
    s.theta = th.ctypes.data_as(C.POINTER(C.c_double))
    s.time = tt.ctypes.data_as(C.POINTER(C.c_double))
    return s


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


class Context:
    """One libdinr context: geometry, network shape, sampling, B, workspace."""

    def __init__(self, geom, mlp_spec, sampling, B: np.ndarray, precision: int = FP32,
                 workspace_bytes: int = 1 << 30, recompute: bool = False):
        L = load()
        keep: list = []
        g = _geometry(geom, keep)
        m = MLP()
        m.n_freq, m.width, m.depth = mlp_spec.n_freq, mlp_spec.width, mlp_spec.depth
        m.act, m.out_act, m.precision, m.mu0 = mlp_spec.act, mlp_spec.out_act, precision, mlp_spec.mu0
        m.recompute = 1 if recompute else 0
        s = Sampling()
        s.mode, s.n, s.n_min, s.n_max, s.h = (sampling.mode, sampling.n, sampling.n_min,
                                              sampling.n_max, sampling.h)
        s.sub = getattr(sampling, "sub", 1)
        s.jitter = getattr(sampling, "jitter", 0)
        s.seed = getattr(sampling, "seed", 0)
        Bh = np.ascontiguousarray(np.asarray(B, dtype=np.float32))
        h = C.c_void_p()
        rc = L.dinr_create(C.byref(g), C.byref(m), C.byref(s),
                           Bh.ctypes.data_as(C.POINTER(C.c_float)), int(workspace_bytes),
                           C.byref(h))
        if rc != OK:
            raise DinrError(rc, "dinr_create rejected the description")
        self._h = h
        self._lib = L
        self.n_params = int(L.dinr_num_params(h))
        self.precision = precision

    def close(self):
        if getattr(self, "_h", None):
            self._lib.dinr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int):
        if rc != OK:
            raise DinrError(rc, self._lib.dinr_last_error(self._h).decode())

    def set_sample_epoch(self, epoch: int):
        """Key word of the random sample positions for the following calls."""
        self._check(self._lib.dinr_set_sample_epoch(self._h, int(epoch) & 0xFFFFFFFF))

    def forward_project(self, params, idx, proj=None, n_out=None):
        """pbar [R] (FP32 device tensor) for projection indices idx (int64)."""
        import torch
        R = idx.shape[0]
        if proj is None:
            proj = torch.empty(R, dtype=torch.float32, device=idx.device)
        self._check(self._lib.dinr_forward_project(self._h, _ptr(params), _ptr(idx), R, _ptr(proj),
                                                   _ptr(n_out), _stream()))
        return proj

    def forward_project_noalloc(self, params, idx, proj, n_out=None):
        """forward_project with the library's static scratch: allocates
        nothing, so proj (and n_out) must be given."""
        self._check(self._lib.dinr_forward_project_noalloc(self._h, _ptr(params), _ptr(idx),
                                                           idx.shape[0], _ptr(proj), _ptr(n_out),
                                                           _stream()))
        return proj

    def project_backward(self, params, idx, dproj, grad=None, gnorm=None):
        import torch
        if grad is None:
            grad = torch.empty(self.n_params, dtype=torch.float32, device=params.device)
        self._check(self._lib.dinr_project_backward(self._h, _ptr(params), _ptr(idx), idx.shape[0],
                                                    _ptr(dproj), _ptr(grad), _ptr(gnorm),
                                                    _stream()))
        return grad

    def step(self, params, idx, meas, grad=None, proj=None, loss=None, gnorm=None, adam=None):
        """One training step; returns (grad, proj, loss, gnorm) device tensors.
        adam = (m, v, lr, beta1, beta2, eps, step) updates params in place."""
        import torch
        dev = params.device
        if grad is None:
            grad = torch.empty(self.n_params, dtype=torch.float32, device=dev)
        if loss is None:
            loss = torch.empty(1, dtype=torch.float64, device=dev)
        if gnorm is None:
            gnorm = torch.empty(1, dtype=torch.float64, device=dev)
        ad = None
        if adam is not None:
            m, v, lr, b1, b2, eps, k = adam
            ad = Adam(m.data_ptr(), v.data_ptr(), lr, b1, b2, eps, int(k))
        self._check(self._lib.dinr_step(self._h, _ptr(params), _ptr(idx), idx.shape[0], _ptr(meas),
                                        _ptr(proj), _ptr(grad), _ptr(loss), _ptr(gnorm),
                                        C.byref(ad) if ad is not None else None, _stream()))
        return grad, proj, loss, gnorm

    def step_status(self) -> int:
        return int(self._lib.dinr_step_status(self._h, _stream()))

    def profile(self, enable: bool = True):
        self._check(self._lib.dinr_profile_enable(self._h, 1 if enable else 0))

    def profile_read(self, kind: int):
        """(total milliseconds, launches) of one kernel class since the last read."""
        t = C.c_double()
        n = C.c_int64()
        self._check(self._lib.dinr_profile_read(self._h, kind, C.byref(t), C.byref(n)))
        return t.value, n.value


class Server:
    """Continuously batched queries of a trained field (slices, reprojections)."""

    def __init__(self, ctx: "Context", params, mem_budget: int = 1 << 30, max_active: int = 64):
        self._ctx = ctx
        self._params = params  # must stay alive and unchanged
        h = C.c_void_p()
        ctx._check(ctx._lib.dinr_server_create(ctx._h, _ptr(params), int(mem_budget),
                                               int(max_active), C.byref(h)))
        self._h = h
        self._lib = ctx._lib

    def submit(self, kind: int, n: int, z_or_theta: float, t: float, out,
               samples_per_ray: int = 0) -> int:
        r = Request(kind, n, z_or_theta, t, samples_per_ray, 0)
        tk = C.c_uint64()
        self._ctx._check(self._lib.dinr_query(self._h, C.byref(r), _ptr(out), C.byref(tk)))
        return tk.value

    def poll(self, ticket: int):
        """(done, latency_ms)."""
        d = C.c_int32()
        lat = C.c_double()
        self._ctx._check(self._lib.dinr_poll(self._h, ticket, C.byref(d), C.byref(lat)))
        return bool(d.value), lat.value

    def wait(self, ticket: int):
        self._ctx._check(self._lib.dinr_query_wait(self._h, ticket))

    def release(self, ticket: int):
        self._ctx._check(self._lib.dinr_query_release(self._h, ticket))

    def write_volume(self, path: str, n: int, nz: int, times, slots: int = 0) -> dict:
        """The field on an n x n x nz grid at each time in `times`, streamed to
        `path` (layout: see dinr_volume_write)."""
        tt = (C.c_double * len(times))(*[float(t) for t in times])
        v = Volume(int(n), int(nz), len(times), int(slots), tt)
        st = VolumeStats()
        self._ctx._check(self._lib.dinr_volume_write(self._h, C.byref(v), path.encode(),
                                                     C.byref(st)))
        return dict(bytes=st.bytes, seconds=st.seconds, voxels_per_s=st.voxels_per_s)

    def stats(self):
        a, b, c, d, e = C.c_int64(), C.c_int64(), C.c_size_t(), C.c_int32(), C.c_int32()
        self._ctx._check(self._lib.dinr_server_stats(self._h, C.byref(a), C.byref(b), C.byref(c),
                                                     C.byref(d), C.byref(e)))
        return dict(launches=a.value, tiles=b.value, bytes_in_use=c.value, queued=d.value,
                    admitted=e.value)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.dinr_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def probe_mfma(kind: int, iters: int) -> float:
    """Sustained BF16 matrix-core rate in TFLOP/s on the current device:
    kind 0 register operands, kind 1 A operand from LDS (dinr_probe_mfma)."""
    lib = load()
    t = C.c_double(0.0)
    rc = lib.dinr_probe_mfma(int(kind), int(iters), _stream(), C.byref(t))
    if rc != 0:
        raise DinrError(rc, "dinr_probe_mfma failed")
    return t.value


def project_function():
    """torch.autograd.Function: pbar = forward_project(params); its backward
    is the library's adjoint (Eq. (8) with the incoming gradient)."""
    import torch

    class DinrProject(torch.autograd.Function):
        @staticmethod
        def forward(ctx, params, idx, dctx):
            ctx.save_for_backward(params, idx)
            ctx.dctx = dctx
            return dctx.forward_project(params.detach().contiguous(), idx)

        @staticmethod
        def backward(ctx, gproj):
            params, idx = ctx.saved_tensors
            g = ctx.dctx.project_backward(params.detach().contiguous(), idx,
                                          gproj.detach().contiguous().float())
            return g, None, None

    return DinrProject
