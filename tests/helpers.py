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
