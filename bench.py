"""Benchmark of one DINR training step on one MI355X.

A step is the whole hot path over one batch of synthetic rays: ray setup,
sampling, Fourier encoding, the MLP forward, the ray-sum, the FP64 loss, the
hand-written adjoint, the weight-gradient reduction and the Adam update.
The headline workload is the BF16 matrix-core path on the 65,536-ray x
256-sample parallel-beam batch (c2); the FP32 path on the same inputs (c1) is
timed beside it and the differences between the two are reported.

Prints one JSON line (see the keys below).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"bf16": 2.5e15, "fp32": 157.3e12}  # dense matrix-core FLOP/s, MI355X datasheet


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_workload(name, prec, batch, steps, warmup, ws_bytes):
    import torch
    from paper_2404_19075_amd import dinr
    w = batch.workload
    ctx = dinr.Context(w.geom, w.mlp, w.sampling, batch.B, precision=prec,
                       workspace_bytes=ws_bytes)
    dev = torch.device("cuda:0")
    P = torch.tensor(batch.params, device=dev)
    idx = torch.tensor(batch.idx, device=dev)
    meas = torch.tensor(batch.meas, device=dev)
    grad = torch.empty(ctx.n_params, device=dev)
    proj = torch.empty(len(batch.idx), device=dev)
    loss = torch.empty(1, dtype=torch.float64, device=dev)
    gnorm = torch.empty(1, dtype=torch.float64, device=dev)
    m = torch.zeros(ctx.n_params, device=dev)
    v = torch.zeros(ctx.n_params, device=dev)
    P0 = P.clone()
    # un-timed reference step (gradient at the initial parameters, no Adam)
    ctx.step(P0, idx, meas, grad=grad, proj=proj, loss=loss, gnorm=gnorm)
    torch.cuda.synchronize()
    ref = dict(grad=grad.cpu().numpy().copy(), proj=proj.cpu().numpy().copy(),
               loss=float(loss.item()))
    k = 0
    for _ in range(warmup):
        k += 1
        ctx.step(P, idx, meas, grad=grad, proj=proj, loss=loss, gnorm=gnorm,
                 adam=(m, v, 1e-3, 0.9, 0.999, 1e-8, k))
    torch.cuda.synchronize()
    ctx.profile(True)
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    for _ in range(steps):
        k += 1
        ctx.step(P, idx, meas, grad=grad, proj=proj, loss=loss, gnorm=gnorm,
                 adam=(m, v, 1e-3, 0.9, 0.999, 1e-8, k))
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    kern = {}
    for kind, kname in [(dinr.PROF_MLP_FWD, "mlp_fwd"), (dinr.PROF_MLP_BWD, "mlp_bwd"),
                        (dinr.PROF_MLP_FUSED, "mlp_fused"), (dinr.PROF_WGRAD, "wgrad")]:
        t, n = ctx.profile_read(kind)
        if n:
            kern[kname] = dict(total_ms=t, launches=n, ms_per_step=t / steps)
    status = ctx.step_status()
    ctx.close()
    del P, idx, meas, grad, proj, m, v, P0
    torch.cuda.empty_cache()
    return ms, kern, ref, status


def cpu_baseline(batch, n_rays=192):
    """The FP64 oracle as it stands, on a bounded ray subset of the same batch."""
    from oracle import oracle as O
    w = batch.workload
    sub = slice(0, n_rays)
    O.build(force=False)
    threads = O.threads()
    t0 = time.perf_counter()
    O.step(w.geom, w.mlp, w.sampling, batch.B, batch.params, batch.idx[sub], batch.meas[sub])
    dt = time.perf_counter() - t0
    samples = n_rays * w.sampling.n
    return dict(value=samples / dt, unit="ray-samples/s", cores=threads, kind="oracle",
                sample=f"{n_rays} rays x {w.sampling.n} samples of the same batch, forward + "
                       f"adjoint in FP64 ({dt:.1f} s)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 comparison run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--workspace-gb", type=float, default=120.0)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU's share of the batch; this build has no multi-GPU "
              "path (the step would shard by one gradient all-reduce, see DESIGN.md).",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2404_19075_amd import dinr
    from paper_2404_19075_amd import synth as S
    dinr.load()
    t0 = time.perf_counter()
    batch = S.make_batch("c2")
    w = batch.workload
    P_pts = len(batch.idx) * w.sampling.n
    log(f"inputs ready in {time.perf_counter() - t0:.1f} s: R={len(batch.idx)} points={P_pts}")
    ws = int(args.workspace_gb * (1 << 30))

    ms_bf16, kern, ref_bf16, status = run_workload("c2", dinr.BF16, batch, args.steps,
                                                   args.warmup, ws)
    log(f"bf16 step {ms_bf16:.3f} ms  kernels {json.dumps(kern)}  status {status}")
    fp32 = None
    if not args.no_fp32:
        ms_fp32, kern32, ref_fp32, _ = run_workload("c1", dinr.FP32, batch, max(2, args.steps // 4),
                                                    1, ws)
        log(f"fp32 step {ms_fp32:.3f} ms  kernels {json.dumps(kern32)}")

        def rel(a, b):
            return float(np.linalg.norm(a.astype(np.float64) - b) / np.linalg.norm(b))
        fp32 = dict(ms_per_step=ms_fp32, value=P_pts / (ms_fp32 * 1e-3),
                    bf16_vs_fp32_rel_err=dict(
                        proj=rel(ref_bf16["proj"], ref_fp32["proj"].astype(np.float64)),
                        grad=rel(ref_bf16["grad"], ref_fp32["grad"].astype(np.float64)),
                        loss=abs(ref_bf16["loss"] - ref_fp32["loss"]) / ref_fp32["loss"]),
                    kernels=kern32)

    spec = w.mlp
    f_fwd = spec.fwd_flops_per_point()
    f_all = spec.flops_per_point()
    shapes = spec.layer_shapes()
    f_dx = sum(2 * o * i for o, i in shapes[1:])
    f_dw = sum(2 * o * i for o, i in shapes[:-1])
    # algorithmic FLOP per launch of each kernel class (per step: one launch of
    # the forward, one backward launch per stash chunk, one wgrad launch per
    # layer and chunk)
    alg = {"mlp_fwd": f_fwd * P_pts, "mlp_bwd": (f_dx + 2 * shapes[-1][1]) * P_pts,
           "mlp_fused": (f_fwd + f_dx + 2 * shapes[-1][1]) * P_pts, "wgrad": f_dw * P_pts}
    dom = max(kern, key=lambda k: kern[k]["ms_per_step"])
    ach = alg[dom] / (kern[dom]["ms_per_step"] * 1e-3)
    roof = dict(bound="mfma", kernel=dom, achieved=ach / 1e12, peak=PEAK["bf16"] / 1e12,
                unit="TFLOP/s", frac=ach / PEAK["bf16"], traffic=None,
                kernels={k: dict(ms_per_step=kern[k]["ms_per_step"],
                                 alg_tflops=alg[k] / (kern[k]["ms_per_step"] * 1e-3) / 1e12)
                         for k in kern},
                step_frac=(f_all * P_pts / (ms_bf16 * 1e-3)) / PEAK["bf16"])
    cpu = None if args.no_cpu else cpu_baseline(batch)
    out = {
        "metric": "ray-samples/s fwd+bwd (one training step incl. Adam), BF16 matrix cores",
        "value": P_pts / (ms_bf16 * 1e-3),
        "unit": "ray-samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_bf16,
        "steps_per_s": 1e3 / ms_bf16,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "c2: parallel beam 256x256 detector, 720 views over 360 deg, "
                               "65536 rays x 256 samples, GRFF 2C=256, 6 ReLU layers of width "
                               "256, softplus output, BF16 MLP GEMMs",
                   "rays": len(batch.idx), "samples_per_ray": w.sampling.n,
                   "ray_samples": P_pts, "flop_per_sample": f_all},
        "fp32": fp32,
        "roofline": roof,
        "cpu_baseline": cpu,
        "status": status,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
