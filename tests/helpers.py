"""Shared helpers of the GPU parity tests: build a libdinr context and the
matching oracle inputs from one seeded synthetic workload."""
from __future__ import annotations

import dataclasses
import sys

import numpy as np

from paper_2404_19075_amd import synth as S


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(x, ref) -> float:
    """Norm-wise relative error ||x - ref||_2 / ||ref||_2."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = np.linalg.norm(ref)
    return float(np.linalg.norm(x - ref) / (d if d > 0 else 1.0))


def param_slices(spec: S.MLPSpec):
    """(name, slice) of every tensor in the flat parameter layout."""
    out = []
    o = 0
    fin = 2 * spec.n_freq
    for l in range(spec.depth):
        n = spec.width * fin
        out.append((f"W{l + 1}", slice(o, o + n)))
        o += n
        out.append((f"b{l + 1}", slice(o, o + spec.width)))
        o += spec.width
        fin = spec.width
    out.append(("w_o", slice(o, o + spec.width)))
    o += spec.width
    out.append(("b_o", slice(o, o + 1)))
    return out


def grad_errors(w, g, ref):
    """Norm-wise relative error of every parameter tensor, and of the whole
    gradient."""
    errs = {name: rel(g[sl], ref[sl]) for name, sl in param_slices(w.mlp)}
    errs["all"] = rel(g, ref)
    return errs


def check_grad(w, g, ref, tol, label):
    """Logs every tensor's error, then holds each to `tol` (a float, or a
    dict: 'first' for the first layer's W and b, 'rest' for the other
    tensors, 'all' for the whole gradient)."""
    errs = grad_errors(w, g, ref)
    log(f"  {label}: " + " ".join(f"{k} {v:.2e}" for k, v in errs.items()))
    if not isinstance(tol, dict):
        tol = dict(first=tol, rest=tol, all=tol)
    for name, e in errs.items():
        bound = tol["all"] if name == "all" else tol["first"] if name in ("W1", "b1") \
            else tol["rest"]
        assert e <= bound, (label, name, e, bound)
    return errs["all"]


def small_workload(name: str, n_rays: int, **kw) -> S.Workload:
    w = S.workload(name)
    w = dataclasses.replace(w, n_rays=n_rays)
    if kw:
        w = dataclasses.replace(w, **kw)
    return w


def device_inputs(batch: S.Batch, dev="cuda"):
    import torch
    return (torch.tensor(batch.params, device=dev),
            torch.tensor(batch.idx, device=dev),
            torch.tensor(batch.meas, device=dev))


def make_ctx(w: S.Workload, B: np.ndarray, precision: int, ws_bytes: int = 2 << 30,
             recompute: bool = False):
    from paper_2404_19075_amd import dinr
    return dinr.Context(w.geom, w.mlp, w.sampling, B, precision=precision,
                        workspace_bytes=ws_bytes, recompute=recompute)


def near_tie(q) -> np.ndarray:
    """Chord lengths l/h within rounding of an integer: there the FP32 sample
    count ceil(l/h) of the device may differ by one from the oracle's FP64 one."""
    q = np.asarray(q, dtype=np.float64)
    return np.abs(q - np.round(q)) < 1e-4 * np.maximum(q, 1)


def resolve_counts(n_proj_gpu, n_ray_ref, q_ray, D2: int) -> np.ndarray:
    """Per-ray sample counts for the oracle that reproduce the device's
    per-projection totals |Phi_r|: the oracle's own counts, with rays whose
    chord sits on a multiple of the step moved by one where a projection's
    total differs.  Fails unless every difference is explained, uniquely, by
    such near ties."""
    n = np.asarray(n_ray_ref, dtype=np.int32).reshape(-1, D2).copy()
    tie = near_tie(q_ray).reshape(-1, D2)
    n_proj_gpu = np.asarray(n_proj_gpu)
    for r in np.nonzero(n.sum(axis=1) != n_proj_gpu)[0]:
        d = int(n_proj_gpu[r]) - int(n[r].sum())
        cand = np.nonzero(tie[r])[0]
        assert len(cand) == abs(d), (r, d, cand)
        n[r, cand] += 1 if d > 0 else -1
    return n.ravel()
