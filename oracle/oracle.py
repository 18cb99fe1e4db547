"""ctypes front-end of the FP64 oracle (dinr_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may use this module; the product path never does.  It builds
the C oracle with gcc (no fast-math, so IEEE double semantics hold) and
converts the shared input descriptions into the oracle's own structs.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dinr_oracle.c")
LIB = os.path.join(HERE, "_build", "liboracle.so")


def build(force: bool = True) -> str:
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-fno-fast-math", "-ffp-contract=off", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Geom(C.Structure):
    _fields_ = [("kind", C.c_int32), ("rows", C.c_int32), ("cols", C.c_int32),
                ("n_views", C.c_int32), ("fov_kind", C.c_int32), ("pad_", C.c_int32),
                ("sod", C.c_double), ("sdd", C.c_double), ("pitch_u", C.c_double),
                ("pitch_v", C.c_double), ("off_u", C.c_double), ("off_v", C.c_double),
                ("fov", C.c_double * 6), ("t0", C.c_double), ("t1", C.c_double),
                ("theta", C.POINTER(C.c_double)), ("time", C.POINTER(C.c_double))]


class _MLP(C.Structure):
    _fields_ = [("n_freq", C.c_int32), ("width", C.c_int32), ("depth", C.c_int32),
                ("act", C.c_int32), ("out_act", C.c_int32), ("pad_", C.c_int32),
                ("mu0", C.c_double)]


class _Samp(C.Structure):
    _fields_ = [("mode", C.c_int32), ("n", C.c_int32), ("n_min", C.c_int32),
                ("n_max", C.c_int32), ("h", C.c_double), ("sub", C.c_int32),
                ("jitter", C.c_int32), ("seed", C.c_uint32), ("epoch", C.c_uint32)]


class _Field(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_items", C.c_int32), ("data", C.POINTER(C.c_double))]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        L = C.CDLL(LIB)
        P = C.POINTER
        d, i32, i64 = C.c_double, C.c_int32, C.c_int64
        L.orc_ray.argtypes = [P(_Geom), i64, P(d), P(d), P(d)]
        L.orc_ray.restype = C.c_int
        L.orc_subray.argtypes = [P(_Geom), i64, i32, i32, P(d), P(d), P(d)]
        L.orc_subray.restype = C.c_int
        L.orc_philox4x32_10.argtypes = [P(C.c_uint32), P(C.c_uint32), P(C.c_uint32)]
        L.orc_philox4x32_10.restype = None
        L.orc_offset.argtypes = [P(_Samp), i64, i32, i32]
        L.orc_offset.restype = d
        L.orc_clip.argtypes = [P(_Geom), P(d), P(d), P(d), P(d)]
        L.orc_clip.restype = None
        L.orc_nsamp.argtypes = [P(_Samp), d]
        L.orc_nsamp.restype = i32
        L.orc_normalize.argtypes = [P(_Geom), P(d), d, P(d)]
        L.orc_normalize.restype = None
        L.orc_nparams.argtypes = [P(_MLP)]
        L.orc_nparams.restype = i64
        L.orc_forward.argtypes = [P(_Geom), P(_MLP), P(_Samp), P(_Field), P(d), P(d), P(i64), i64,
                                  P(i32), P(d), P(i32), P(d), P(d), C.c_int]
        L.orc_forward.restype = C.c_int
        L.orc_step.argtypes = [P(_Geom), P(_MLP), P(_Samp), P(d), P(d), P(i64), i64, P(d), P(i32),
                               P(d), P(d), P(d), C.c_int]
        L.orc_step.restype = C.c_int
        L.orc_field_points.argtypes = [P(_Geom), P(_MLP), P(d), P(d), P(d), i64, P(d), C.c_int]
        L.orc_field_points.restype = C.c_int
        L.orc_adam.argtypes = [P(d), P(d), P(d), P(d), i64, d, d, d, d, i64]
        L.orc_adam.restype = None
        L.orc_threads.argtypes = []
        L.orc_threads.restype = C.c_int
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class _Keep:
    """Holds converted arrays alive while a struct points into them."""

    def __init__(self):
        self.refs = []

    def f64(self, a) -> np.ndarray:
        a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
        self.refs.append(a)
        return a


def _geom(g, keep: _Keep) -> _Geom:
    th = keep.f64(g.theta)
    tt = keep.f64(g.time)
    s = _Geom()
    s.kind, s.rows, s.cols, s.n_views, s.fov_kind = g.kind, g.rows, g.cols, g.n_views, g.fov_kind
    s.sod, s.sdd = g.sod, g.sdd
    s.pitch_u, s.pitch_v, s.off_u, s.off_v = g.pitch_u, g.pitch_v, g.off_u, g.off_v
    for k in range(6):
        s.fov[k] = g.fov[k] if k < len(g.fov) else 0.0
    s.t0, s.t1 = g.t0, g.t1
    s.theta, s.time = _dp(th), _dp(tt)
    return s


def _mlp(m) -> _MLP:
    s = _MLP()
    s.n_freq, s.width, s.depth, s.act, s.out_act, s.mu0 = (m.n_freq, m.width, m.depth, m.act,
                                                           m.out_act, m.mu0)
    return s


def _samp(sp) -> _Samp:
    s = _Samp()
    s.mode, s.n, s.n_min, s.n_max, s.h = sp.mode, sp.n, sp.n_min, sp.n_max, sp.h
    s.sub = getattr(sp, "sub", 1)
    s.jitter = getattr(sp, "jitter", 0)
    s.seed = getattr(sp, "seed", 0)
    s.epoch = getattr(sp, "epoch", 0)
    return s


def sub_rays(sp) -> int:
    """Rays per projection, D^2."""
    D = max(1, getattr(sp, "sub", 1))
    return D * D


def threads() -> int:
    return lib().orc_threads()


def nparams(m) -> int:
    return int(lib().orc_nparams(C.byref(_mlp(m))))


def ray(g, i: int):
    keep = _Keep()
    o, d, t = np.zeros(3), np.zeros(3), np.zeros(1)
    rc = lib().orc_ray(C.byref(_geom(g, keep)), int(i), _dp(o), _dp(d), _dp(t))
    if rc != 0:
        raise IndexError(i)
    return o, d, float(t[0])


def philox4x32_10(ctr, key):
    """Philox4x32-10 of a 4-word counter under a 2-word key (4 uint32 words)."""
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    out = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, out)
    return [int(v) for v in out]


def offset(sp, i: int, k: int, j: int) -> float:
    """Position in [0, 1) of sample j of ray k of projection i in its segment."""
    return float(lib().orc_offset(C.byref(_samp(sp)), int(i), int(k), int(j)))


def subray(g, i: int, D: int, k: int):
    """Ray k = b D + a of projection i: to the centre of sub-pixel (b, a)."""
    keep = _Keep()
    o, d, t = np.zeros(3), np.zeros(3), np.zeros(1)
    rc = lib().orc_subray(C.byref(_geom(g, keep)), int(i), int(D), int(k), _dp(o), _dp(d),
                          _dp(t))
    if rc != 0:
        raise IndexError((i, D, k))
    return o, d, float(t[0])


def clip(g, o, d):
    keep = _Keep()
    o = keep.f64(o)
    d = keep.f64(d)
    si, ln = np.zeros(1), np.zeros(1)
    lib().orc_clip(C.byref(_geom(g, keep)), _dp(o), _dp(d), _dp(si), _dp(ln))
    return float(si[0]), float(ln[0])


def nsamp(sp, length: float) -> int:
    return int(lib().orc_nsamp(C.byref(_samp(sp)), float(length)))


def normalize(g, x, t):
    keep = _Keep()
    x = keep.f64(x)
    r = np.zeros(4)
    lib().orc_normalize(C.byref(_geom(g, keep)), _dp(x), float(t), _dp(r))
    return r


def forward(g, m, sp, B, params, idx, field: Optional[tuple] = None,
            n_override: Optional[np.ndarray] = None, nthreads: int = 0):
    """pbar [R] (float64), and n, s_in, l of every ray, [R D^2] (ray k of
    projection r at r D^2 + k).  field = (kind, data[n,k]) replaces the MLP by
    an analytic field; n_override is [R D^2]."""
    keep = _Keep()
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
    R = idx.shape[0]
    RS = R * sub_rays(sp)
    Bd = keep.f64(B if B is not None else np.zeros((1, 4)))
    Pd = keep.f64(params if params is not None else np.zeros(1))
    proj, si, ln = np.zeros(R), np.zeros(RS), np.zeros(RS)
    n = np.zeros(RS, dtype=np.int32)
    fs = None
    if field is not None:
        kind, data = field
        data = keep.f64(np.asarray(data, dtype=np.float64).ravel())
        fs = _Field()
        fs.kind = int(kind)
        fs.n_items = int(len(np.atleast_2d(field[1]))) if kind in (2, 3) else 1
        fs.data = _dp(data)
    nov = None
    if n_override is not None:
        nov = np.ascontiguousarray(np.asarray(n_override, dtype=np.int32))
        assert nov.shape == (RS,), "n_override holds one count per ray"
        keep.refs.append(nov)
    rc = lib().orc_forward(C.byref(_geom(g, keep)), C.byref(_mlp(m)), C.byref(_samp(sp)),
                           C.byref(fs) if fs is not None else None, _dp(Bd), _dp(Pd),
                           idx.ctypes.data_as(C.POINTER(C.c_int64)), R,
                           nov.ctypes.data_as(C.POINTER(C.c_int32)) if nov is not None else None,
                           _dp(proj), n.ctypes.data_as(C.POINTER(C.c_int32)), _dp(si), _dp(ln),
                           int(nthreads))
    if rc != 0:
        raise RuntimeError("orc_forward failed")
    return proj, n, si, ln


def step(g, m, sp, B, params, idx, meas, n_override=None, nthreads: int = 0):
    """(loss, grad [n_params], pbar [R]) in float64 (Eqs. (5) and (8))."""
    keep = _Keep()
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
    R = idx.shape[0]
    Bd, Pd, Md = keep.f64(B), keep.f64(params), keep.f64(meas)
    grad = np.zeros(Pd.shape[0])
    proj = np.zeros(R)
    loss = np.zeros(1)
    nov = None
    if n_override is not None:
        nov = np.ascontiguousarray(np.asarray(n_override, dtype=np.int32))
        assert nov.shape == (R * sub_rays(sp),), "n_override holds one count per ray"
        keep.refs.append(nov)
    rc = lib().orc_step(C.byref(_geom(g, keep)), C.byref(_mlp(m)), C.byref(_samp(sp)), _dp(Bd),
                        _dp(Pd), idx.ctypes.data_as(C.POINTER(C.c_int64)), R, _dp(Md),
                        nov.ctypes.data_as(C.POINTER(C.c_int32)) if nov is not None else None,
                        _dp(proj), _dp(grad), _dp(loss), int(nthreads))
    if rc != 0:
        raise RuntimeError("orc_step failed")
    return float(loss[0]), grad, proj


def field_points(g, m, B, params, pts, nthreads: int = 0) -> np.ndarray:
    """mu0 * M at world points [n,4] = (x, y, z, t)."""
    keep = _Keep()
    pts = keep.f64(pts).reshape(-1, 4)
    out = np.zeros(pts.shape[0])
    rc = lib().orc_field_points(C.byref(_geom(g, keep)), C.byref(_mlp(m)), _dp(keep.f64(B)),
                                _dp(keep.f64(params)), _dp(pts), pts.shape[0], _dp(out),
                                int(nthreads))
    if rc != 0:
        raise RuntimeError("orc_field_points failed")
    return out


def adam(params, grad, m, v, lr, b1, b2, eps, step_idx):
    """In-place Adam on float64 arrays."""
    for a in (params, grad, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    lib().orc_adam(_dp(params), _dp(grad), _dp(m), _dp(v), params.shape[0], lr, b1, b2, eps,
                   int(step_idx))
