"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/dinr.h declares, and rejects invalid descriptions with
DINR_EINVAL before touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2404_19075_amd import dinr
from paper_2404_19075_amd import synth as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dinr.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(dinr_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["dinr_create", "dinr_destroy", "dinr_forward_project", "dinr_project_backward",
              "dinr_step", "dinr_last_error"]:
        assert n in names
    assert set(names) == set(dinr.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(dinr.LIB_PATH)
    for n in declared_functions():
        assert hasattr(lib, n), n


def _create(geom=None, mlp=None, samp=None, B=None, budget=64 << 20):
    w = S.workload("c0")
    g = geom or w.geom
    m = mlp or w.mlp
    sp = samp or w.sampling
    B = S.make_B(m, 0) if B is None else B
    L = dinr.load()
    keep = []
    gs = dinr._geometry(g, keep)
    ms = dinr.MLP()
    ms.n_freq, ms.width, ms.depth, ms.act, ms.out_act, ms.precision, ms.mu0 = (
        m.n_freq, m.width, m.depth, m.act, m.out_act, getattr(m, "precision", 0), m.mu0)
    ss = dinr.Sampling()
    ss.mode, ss.n, ss.n_min, ss.n_max, ss.h = sp.mode, sp.n, sp.n_min, sp.n_max, sp.h
    ss.sub, ss.jitter, ss.seed = sp.sub, sp.jitter, sp.seed
    Bh = np.ascontiguousarray(B, dtype=np.float32)
    h = C.c_void_p()
    rc = L.dinr_create(C.byref(gs), C.byref(ms), C.byref(ss),
                       Bh.ctypes.data_as(C.POINTER(C.c_float)), budget, C.byref(h))
    return rc, h


def _replace(obj, **kw):
    import dataclasses
    return dataclasses.replace(obj, **kw)


@pytest.mark.parametrize("change", [
    dict(geom=dict(kind=7)),
    dict(geom=dict(rows=0)),
    dict(geom=dict(pitch_u=0.0)),
    dict(geom=dict(fov=(1, -1, -1, 1, -1, 1))),
    dict(geom=dict(fov_kind=3)),
    dict(geom=dict(t0=1.0, t1=1.0)),
    dict(geom=dict(kind=1, sod=10.0, sdd=5.0)),
    dict(mlp=dict(width=96)),
    dict(mlp=dict(depth=0)),
    dict(mlp=dict(depth=11)),
    dict(mlp=dict(act=2)),
    dict(mlp=dict(out_act=5)),
    dict(samp=dict(n=0)),
    dict(samp=dict(mode=1, h=0.0)),
    dict(samp=dict(mode=1, h=0.01, n_min=10, n_max=5)),
    dict(samp=dict(sub=9)),
    dict(samp=dict(sub=-1)),
    dict(samp=dict(jitter=2)),
])
def test_create_rejects_invalid_descriptions(change):
    w = S.workload("c0")
    g = _replace(w.geom, **change.get("geom", {}))
    m = _replace(w.mlp, **change.get("mlp", {}))
    sp = _replace(w.sampling, **change.get("samp", {}))
    rc, h = _create(g, m, sp)
    assert rc == dinr.EINVAL and not h.value


def test_create_rejects_nonfinite_B_and_small_budget():
    w = S.workload("c0")
    B = S.make_B(w.mlp, 0)
    B[3, 2] = np.nan
    rc, h = _create(B=B)
    assert rc == dinr.EINVAL
    rc, h = _create(budget=1 << 20)
    assert rc == dinr.ENOMEM


def test_null_arguments():
    L = dinr.load()
    assert L.dinr_create(None, None, None, None, 0, None) == dinr.EINVAL
    assert L.dinr_forward_project(None, None, None, 0, None, None, None) == dinr.EINVAL
    assert L.dinr_step(None, None, None, 0, None, None, None, None, None, None, None) == dinr.EINVAL
    assert L.dinr_destroy(None) == dinr.OK
    assert L.dinr_volume_write(None, None, None, None) == dinr.EINVAL
    assert L.dinr_set_sample_epoch(None, 3) == dinr.EINVAL
