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
PEAK_HBM = 8.0e12  # B/s, MI355X datasheet


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# per-step time statistics of each timed leg (median, p90, extremes)
STEP_STATS = {}


def run_workload(name, prec, batch, steps, warmup, ws_bytes):
    """Times `steps` training steps (Adam included) after `warmup` untimed ones.
    Returns (ms per step, per-kernel times, the un-timed reference step's
    outputs, the step status, the trained parameters, the batch's ray-samples
    as the device counts them)."""
    import torch
    from paper_2404_19075_amd import dinr
    w = batch.workload
    ctx = dinr.Context(w.geom, w.mlp, w.sampling, batch.B, precision=prec,
                       workspace_bytes=ws_bytes, recompute=bool(getattr(w, "recompute", False)))
    dev = torch.device("cuda:0")
    P = torch.tensor(batch.params, device=dev)
    idx = torch.tensor(batch.idx, device=dev)
    meas = torch.tensor(batch.meas, device=dev)
    # |Phi| of every projection: the ray-samples one step evaluates
    n_out = torch.empty(len(batch.idx), dtype=torch.int32, device=dev)
    ctx.forward_project(P, idx, n_out=n_out)
    torch.cuda.synchronize()
    points = int(n_out.sum().item())
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
    jitter = getattr(w.sampling, "jitter", 0)
    for _ in range(warmup):
        k += 1
        if jitter:
            ctx.set_sample_epoch(k)  # new random sample positions every step
        ctx.step(P, idx, meas, grad=grad, proj=proj, loss=loss, gnorm=gnorm,
                 adam=(m, v, 1e-3, 0.9, 0.999, 1e-8, k))
    torch.cuda.synchronize()
    ctx.profile(True)
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    # an event after every step (no synchronisation between steps): the
    # per-step times give the median and p90 beside the mean
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    e0.record(st)
    for i in range(steps):
        k += 1
        if jitter:
            ctx.set_sample_epoch(k)
        ctx.step(P, idx, meas, grad=grad, proj=proj, loss=loss, gnorm=gnorm,
                 adam=(m, v, 1e-3, 0.9, 0.999, 1e-8, k))
        ev[i].record(st)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    per = [e0.elapsed_time(ev[0])] + [ev[i - 1].elapsed_time(ev[i]) for i in range(1, steps)]
    STEP_STATS[name] = dict(median_ms=float(np.median(per)), p90_ms=float(np.percentile(per, 90)),
                            min_ms=float(min(per)), max_ms=float(max(per)))
    kern = {}
    for kind, kname in [(dinr.PROF_MLP_FWD, "mlp_fwd"), (dinr.PROF_MLP_BWD, "mlp_bwd"),
                        (dinr.PROF_MLP_FUSED, "mlp_fused"), (dinr.PROF_WGRAD, "wgrad"),
                        (dinr.PROF_RAYS, "ray_setup"), (dinr.PROF_LOSS, "loss"),
                        (dinr.PROF_REDUCE, "reduce")]:
        t, n = ctx.profile_read(kind)
        if n:
            kern[kname] = dict(total_ms=t, launches=n, ms_per_step=t / steps,
                               launches_per_step=n / steps)
    status = ctx.step_status()
    trained = P.cpu().numpy()
    ctx.close()
    del P, idx, meas, grad, proj, m, v, P0, n_out
    torch.cuda.empty_cache()
    return ms, kern, ref, status, trained, points


def serving(batch, params_np, n_req=1000, rates=(0.1, 0.5, 1.0, 2.0), n_cap=200, seed=7):
    """Continuously batched queries of the trained field (BF16): a 50/50 mix of
    n x n slices (n in 64..512) at random (z, t) and parallel-beam
    reprojections (n in 128..512, 256 samples per ray) at random (theta, t).
    Capacity is the completion rate of a closed batch of n_cap mixed requests
    submitted at once; then, at each rate (a fraction of that capacity),
    n_req requests arrive as a Poisson stream, each with its own output
    buffer, and the server admits them by its 1 GB output budget and 64 slots.
    Returns capacity and p50/p99 submit-to-completion latency per rate."""
    import torch
    from paper_2404_19075_amd import dinr
    w = batch.workload
    ctx = dinr.Context(w.geom, w.mlp, w.sampling, batch.B, precision=dinr.BF16,
                       workspace_bytes=64 << 20)
    P = torch.tensor(params_np, device="cuda")
    srv = dinr.Server(ctx, P, mem_budget=1 << 30, max_active=64)
    rng = np.random.default_rng(seed)
    pool = [torch.empty(512 * 512, device="cuda") for _ in range(max(n_req, n_cap))]

    def draw():
        if rng.random() < 0.5:
            return (dinr.QUERY_SLICE, int(rng.choice([64, 128, 256, 512])),
                    float(rng.uniform(-1, 1)), float(rng.uniform(0, 1)), 0)
        return (dinr.QUERY_REPROJECTION, int(rng.choice([128, 256, 384, 512])),
                float(rng.uniform(0, 2 * np.pi)), float(rng.uniform(0, 1)), 256)

    def submit(k, r):
        return srv.submit(r[0], r[1], r[2], r[3], pool[k], samples_per_ray=r[4])

    # warm-up, then capacity: a closed batch of mixed requests submitted at once
    for tk in [submit(k, draw()) for k in range(8)]:
        srv.wait(tk)
        srv.release(tk)
    reqs = [draw() for _ in range(n_cap)]
    st0 = srv.stats()
    t0 = time.perf_counter()
    tks = [submit(k, r) for k, r in enumerate(reqs)]
    for tk in tks:
        srv.wait(tk)
    span = time.perf_counter() - t0
    cap = len(reqs) / span
    st1 = srv.stats()
    for tk in tks:
        srv.release(tk)
    # forward FLOP the batch made the matrix cores do: every point of every
    # tile run (256 points per tile, padding and rays outside the field of
    # view included)
    tiles = st1["tiles"] - st0["tiles"]
    fwd_flop = tiles * 256 * w.mlp.fwd_flops_per_point()
    log(f"serving capacity {cap:.2f} req/s ({n_cap} requests, {tiles} tiles, "
        f"{st1['launches'] - st0['launches']} launches, {fwd_flop / span / 1e12:.0f} TFLOP/s)")
    out = dict(capacity_req_per_s=cap, capacity_requests=n_cap,
               capacity_tiles=tiles, capacity_launches=st1["launches"] - st0["launches"],
               capacity_fwd_tflops=fwd_flop / span / 1e12,
               mix="50% slices n=64..512, 50% reprojections n=128..512 x 256 samples",
               mem_budget_bytes=1 << 30, max_active=64, rates=[])
    for frac in rates:
        rate = frac * cap
        arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n_req))
        pending, kinds = [], []
        start = time.perf_counter()
        for k, a in enumerate(arrivals):
            while time.perf_counter() - start < a:
                time.sleep(0.0002)
            r = draw()
            kinds.append(r[0])
            pending.append(submit(k, r))
            if (k + 1) % 250 == 0:
                log(f"  rate {frac:.2f}x: {k + 1} requests submitted")
        lat = []
        for tk in pending:
            srv.wait(tk)
            lat.append(srv.poll(tk)[1])
            srv.release(tk)
        span = time.perf_counter() - start
        lat = np.array(lat)
        kinds = np.array(kinds)
        row = dict(load=frac, rate_req_per_s=rate, requests=len(lat),
                   p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                   p50_ms_slices=float(np.percentile(lat[kinds == 0], 50)),
                   p99_ms_slices=float(np.percentile(lat[kinds == 0], 99)),
                   p50_ms_reprojections=float(np.percentile(lat[kinds == 1], 50)),
                   p99_ms_reprojections=float(np.percentile(lat[kinds == 1], 99)),
                   throughput_req_per_s=len(lat) / span)
        log(f"serving rate {rate:.2f}/s: {json.dumps(row)}")
        out["rates"].append(row)
    st = srv.stats()
    out["launches"] = st["launches"]
    out["tiles"] = st["tiles"]
    srv.close()
    ctx.close()
    return out


KERNEL_SOURCES = ["dinr_dev.h", "ray_dev.h", "kernels.h", "mlp.h", "mlp_inst.hip", "wgrad.hip",
                  "kernels.hip", "dinr_api.hip"]


def kernel_source_digest():
    """sha256 prefix of the sources that define the step's kernels."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2404_19075_amd", "csrc")
    for name in KERNEL_SOURCES:
        h.update(open(os.path.join(csrc, name), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profile(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by a plain copy's readings), or None
    when the summary was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_c2_bf16.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        parts = line.split()
        if len(parts) == 2 and not line.startswith("#"):
            vals[parts[0]] = parts[1]
    key = f"{kernel}_bytes_per_launch"
    if vals.get("kernel_sources_sha256_16") != kernel_source_digest() or key not in vals:
        return None
    return float(vals[key])


def cpu_baseline(batch, n_rays=1024):
    """The FP64 oracle as it stands, on a bounded ray subset of the same batch."""
    from oracle import oracle as O
    w = batch.workload
    sub = slice(0, n_rays)
    O.build(force=False)
    threads = O.threads()
    # one thread on a smaller subset first, for the per-core rate
    n1 = max(1, n_rays // 16)
    t1 = time.perf_counter()
    O.step(w.geom, w.mlp, w.sampling, batch.B, batch.params, batch.idx[:n1], batch.meas[:n1],
           nthreads=1)
    dt1 = time.perf_counter() - t1
    t0 = time.perf_counter()
    ref = O.step(w.geom, w.mlp, w.sampling, batch.B, batch.params, batch.idx[sub], batch.meas[sub],
                 nthreads=threads)
    dt = time.perf_counter() - t0
    samples = n_rays * w.sampling.n
    full = len(batch.idx) * w.sampling.n
    # the whole tiny workload (c0: 1024 rays x 64 samples, the network of
    # width 64), one full step, on every core and on one
    from paper_2404_19075_amd import synth as S
    b0 = S.make_batch("c0")
    w0 = b0.workload
    c0 = {}
    for label, nt in (("all_cores", threads), ("one_thread", 1)):
        t = time.perf_counter()
        O.step(w0.geom, w0.mlp, w0.sampling, b0.B, b0.params, b0.idx, b0.meas, nthreads=nt)
        dtc = time.perf_counter() - t
        c0[label] = dict(threads=nt, step_s=dtc,
                         ray_samples_per_s=len(b0.idx) * w0.sampling.n / dtc)
    return dict(value=samples / dt, unit="ray-samples/s", cores=threads, kind="oracle",
                sample=f"{n_rays} rays x {w.sampling.n} samples of the same batch, forward + "
                       f"adjoint in FP64 ({dt:.1f} s)",
                one_thread_value=n1 * w.sampling.n / dt1,
                one_thread_sample=f"{n1} rays ({dt1:.1f} s)",
                full_step_s_extrapolated=full / (samples / dt),
                c0_full_step=dict(workload="c0: 1024 rays x 64 samples, GRFF 2C=128, 3 ReLU "
                                           "layers of width 64, forward + adjoint in FP64", **c0)), ref


def errors_vs_oracle(batch, ref, n_rays, ws_bytes):
    """Relative error of the GPU step (BF16 and FP32) against the oracle's
    step on the same ray subset: projections, gradient, loss."""
    import torch
    from paper_2404_19075_amd import dinr
    w = batch.workload
    loss_o, grad_o, proj_o = ref
    out = {"rays": n_rays}
    for name, prec in (("bf16", dinr.BF16), ("fp32", dinr.FP32)):
        ctx = dinr.Context(w.geom, w.mlp, w.sampling, batch.B, precision=prec,
                           workspace_bytes=ws_bytes)
        P = torch.tensor(batch.params, device="cuda")
        idx = torch.tensor(batch.idx[:n_rays], device="cuda")
        meas = torch.tensor(batch.meas[:n_rays], device="cuda")
        pr = torch.empty(n_rays, device="cuda")
        g, _, lo, _ = ctx.step(P, idx, meas, proj=pr)
        torch.cuda.synchronize()

        def rel(a, b):
            return float(np.linalg.norm(a.astype(np.float64) - b) / np.linalg.norm(b))
        out[name] = dict(proj=rel(pr.cpu().numpy(), proj_o), grad=rel(g.cpu().numpy(), grad_o),
                         loss=abs(float(lo.item()) - loss_o) / loss_o)
        ctx.close()
    return out


def inference_volume(batch, params_np, n=256, nz=256, n_times=8):
    """The trained field voxelised on an n x n x nz grid at n_times view times,
    streamed to a temporary file (Sec. IV inference), BF16."""
    import tempfile
    import torch
    from paper_2404_19075_amd import dinr
    w = batch.workload
    ctx = dinr.Context(w.geom, w.mlp, w.sampling, batch.B, precision=dinr.BF16,
                       workspace_bytes=64 << 20)
    P = torch.tensor(params_np, device="cuda")
    srv = dinr.Server(ctx, P, mem_budget=1 << 30, max_active=64)
    times = [float(t) for t in np.asarray(w.geom.time)[:: max(1, len(w.geom.time) // n_times)][:n_times]]
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "volume.bin")
        srv.write_volume(path, 64, 4, times[:1], slots=4)  # warm-up
        st = srv.write_volume(path, n, nz, times, slots=8)
    srv.close()
    ctx.close()
    out = dict(grid=f"{n}x{n}x{nz} at {len(times)} view times", voxels=n * n * nz * len(times),
               bytes=st["bytes"], seconds=st["seconds"], voxels_per_s=st["voxels_per_s"],
               gb_per_s=st["bytes"] / st["seconds"] / 1e9)
    log(f"inference volume: {json.dumps(out)}")
    return out


def stream_rates(kern, R, D2, points, tile=256):
    """HBM rates of the ray and projection streams (GB/s), from the bytes
    each kernel class moves by construction and its HIP-event time.
    ray setup: the projection index (8 B), then per ray record the record
    (64 B) and its count (4 B) written, the count read twice and the point
    offset written by the scan (16 B), and per 256-point tile its first ray
    (4 B).  loss: per projection the measurement and the prediction (4 B
    each) and the upstream gradient written (4 B); the one-pass step's loss
    kernel instead reads each ray record's count and flags (8 B) and the
    measurement (4 B)."""
    out = {}
    n_rec = R * D2
    tiles = (points + tile - 1) // tile
    b = dict(ray_setup=R * 8 + n_rec * (64 + 4 + 16) + tiles * 4, loss=R * 12)
    for k, nbytes in b.items():
        if k in kern:
            ms = kern[k]["ms_per_step"]
            out[k] = dict(ms_per_step=ms, bytes=nbytes, gb_per_s=nbytes / (ms * 1e-3) / 1e9,
                          launches_per_step=kern[k]["launches_per_step"])
    return out


def wgrad_stash_bytes(spec, P_pts, elem=2):
    """Bytes the weight-gradient kernels of one BF16 step read: every byte of
    the adjoint's stash once -- layer 1's point coordinates (16 B) and delta_1,
    h_l and delta_l for the hidden layers, and for the last layer h_{L-1} with
    dL/dz_o (4 B) and the ReLU mask words (one bit per unit) or the Swish
    derivatives -- plus the split partials each launch writes (not counted:
    0.5 % at c2)."""
    hb = spec.width * elem
    L = spec.depth
    per = 16 + (L - 1) * hb + (L - 1) * hb + 4
    per += spec.width // 8 if spec.act == 0 else hb
    return per * P_pts


def alg_flops(spec, P_pts):
    """Algorithmic FLOP per step of each kernel class: the forward GEMMs, the
    adjoint's input-gradient GEMMs (a recomputing backward kernel's repeat of
    the forward is not counted), the weight-gradient GEMMs."""
    f_fwd = spec.fwd_flops_per_point()
    shapes = spec.layer_shapes()
    f_dx = sum(2 * o * i for o, i in shapes[1:])
    f_dw = sum(2 * o * i for o, i in shapes[:-1])
    return {"mlp_fwd": f_fwd * P_pts, "mlp_bwd": (f_dx + 2 * shapes[-1][1]) * P_pts,
            "mlp_fused": (f_fwd + f_dx + 2 * shapes[-1][1]) * P_pts, "wgrad": f_dw * P_pts}


def paper_network(steps, warmup, ws, sub=1, jitter=0):
    """The paper's own network (Swish hidden layers, linear output, five layers
    of width 256) on a c2-sized batch, BF16; optionally with D x D rays per
    projection and stratified random sample positions (App. A, Sec. IV)."""
    import dataclasses
    from paper_2404_19075_amd import dinr
    from paper_2404_19075_amd import synth as S
    w = S.workload("paper")
    w = dataclasses.replace(w, sampling=dataclasses.replace(w.sampling, sub=sub, jitter=jitter,
                                                            seed=17))
    b = S.make_batch(w)
    ms, kern, _, status, _, P_pts = run_workload("paper", dinr.BF16, b, steps, warmup, ws)
    alg = alg_flops(b.workload.mlp, P_pts)
    rays = "65536 projections x 256 samples" if sub == 1 else \
        f"65536 projections x {sub}x{sub} rays x 256 samples, random positions"
    out = dict(workload=f"paper network on the c2 geometry: {rays}, GRFF "
                        "2C=256 (sigma_s 0.5, sigma_t 0.1), 5 Swish layers of width 256, "
                        "linear output, BF16 MLP GEMMs",
               ray_samples=P_pts, ms_per_step=ms, step_ms_stats=STEP_STATS.get("paper"),
               value=P_pts / (ms * 1e-3), unit="ray-samples/s", status=status,
               step_tflops=b.workload.mlp.flops_per_point() * P_pts / (ms * 1e-3) / 1e12,
               kernels={k: dict(ms_per_step=v["ms_per_step"],
                                alg_tflops=alg[k] / (v["ms_per_step"] * 1e-3) / 1e12)
                        for k, v in kern.items() if k in alg},
               other_kernels={k: v for k, v in kern.items() if k not in alg})
    log(f"paper network (D={sub}, jitter={jitter}) step {ms:.3f} ms  {json.dumps(out['kernels'])}")
    return out


def cone_ragged(steps, warmup, ws):
    """The ragged cone-beam workload (c3): 131,072 rays of a 512^2 detector,
    1800 views, n = clamp(ceil(l/h), 32, 512) samples per ray, 8 ReLU layers
    of width 256, BF16, the two-pass step recomputing the forward in the
    backward kernel.  Algorithmic rates leave the recomputed forward out."""
    from paper_2404_19075_amd import dinr
    from paper_2404_19075_amd import synth as S
    t0 = time.perf_counter()
    b = S.make_batch("c3")
    log(f"c3 inputs ready in {time.perf_counter() - t0:.1f} s")
    ms, kern, _, status, _, P_pts = run_workload("c3", dinr.BF16, b, steps, warmup, ws)
    spec = b.workload.mlp
    alg = alg_flops(spec, P_pts)
    f_all = spec.flops_per_point()
    out = dict(workload="c3: cone beam SOD 500 SDD 1000, 512x512 detector, 1800 views over 360 "
                        "deg, 131072 rays x clamp(ceil(l*256), 32, 512) samples, GRFF 2C=256, "
                        "8 ReLU layers of width 256, softplus output, BF16, recomputing backward",
               rays=len(b.idx), ray_samples=P_pts, ms_per_step=ms,
               step_ms_stats=STEP_STATS.get("c3"),
               value=P_pts / (ms * 1e-3), unit="ray-samples/s", status=status,
               step_tflops=f_all * P_pts / (ms * 1e-3) / 1e12,
               step_frac=f_all * P_pts / (ms * 1e-3) / PEAK["bf16"],
               kernels={k: dict(ms_per_step=v["ms_per_step"], launches=v["launches"],
                                alg_tflops=alg[k] / (v["ms_per_step"] * 1e-3) / 1e12,
                                frac=alg[k] / (v["ms_per_step"] * 1e-3) / PEAK["bf16"])
                        for k, v in kern.items() if k in alg},
               streams=stream_rates(kern, len(b.idx), 1, P_pts),
               other_kernels={k: v for k, v in kern.items() if k not in alg})
    log(f"c3 step {ms:.3f} ms  {json.dumps(out['kernels'])}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 comparison run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--workspace-gb", type=float, default=120.0)
    ap.add_argument("--no-serving", action="store_true", help="skip the query-serving run")
    ap.add_argument("--no-paper-net", action="store_true",
                    help="skip the step of the paper's Swish network")
    ap.add_argument("--no-volume", action="store_true",
                    help="skip the 4D inference volume written to disk")
    ap.add_argument("--no-c3", action="store_true", help="skip the ragged cone-beam step")
    ap.add_argument("--serving-requests", type=int, default=1000,
                    help="requests per arrival rate in the serving sweep")
    ap.add_argument("--serving-loads", type=str, default="0.1,0.5,1.0,2.0",
                    help="arrival rates of the serving sweep, as fractions of its capacity")
    ap.add_argument("--copy-calibration", type=float, default=0.0,
                    help="only run a plain device copy of this many GiB (to scale the memory "
                         "counters of a profiler run) and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: there is no multi-GPU path (the step would shard by "
              "drawing an independent batch per GPU and averaging the gradients with one "
              "all-reduce before Adam).", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_calibration > 0:
        n = int(args.copy_calibration * (1 << 30)) // 4
        src = torch.ones(n, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copied {4 * n} bytes")
        return
    from paper_2404_19075_amd import dinr
    from paper_2404_19075_amd import synth as S
    dinr.load()
    t0 = time.perf_counter()
    batch = S.make_batch("c2")
    w = batch.workload
    P_pts = len(batch.idx) * w.sampling.n
    log(f"inputs ready in {time.perf_counter() - t0:.1f} s: R={len(batch.idx)} points={P_pts}")
    ws = int(args.workspace_gb * (1 << 30))

    ms_bf16, kern, ref_bf16, status, trained, P_pts = run_workload("c2", dinr.BF16, batch,
                                                                   args.steps, args.warmup, ws)
    log(f"bf16 step {ms_bf16:.3f} ms  kernels {json.dumps(kern)}  status {status}")
    fp32 = None
    if not args.no_fp32:
        ms_fp32, kern32, ref_fp32, _, _, _ = run_workload("c1", dinr.FP32, batch,
                                                          max(2, args.steps // 4), 1, ws)
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
    f_all = spec.flops_per_point()
    alg = alg_flops(spec, P_pts)
    gemm = {k: v for k, v in kern.items() if k in alg}
    dom = max(gemm, key=lambda k: gemm[k]["ms_per_step"])
    ach = alg[dom] / (kern[dom]["ms_per_step"] * 1e-3)
    roof = dict(bound="mfma", kernel=dom, achieved=ach / 1e12, peak=PEAK["bf16"] / 1e12,
                unit="TFLOP/s", frac=ach / PEAK["bf16"], traffic=None,
                kernels={k: dict(ms_per_step=gemm[k]["ms_per_step"],
                                 alg_tflops=alg[k] / (gemm[k]["ms_per_step"] * 1e-3) / 1e12)
                         for k in gemm},
                step_frac=(f_all * P_pts / (ms_bf16 * 1e-3)) / PEAK["bf16"],
                # the target for the MLP GEMMs: half the dense BF16 peak
                target_frac=0.5, target_met=bool(ach / PEAK["bf16"] >= 0.5),
                streams=stream_rates(kern, len(batch.idx), 1, P_pts),
                other_kernels={k: v for k, v in kern.items() if k not in alg})
    # sustained matrix-core rate of this device: operands in registers, and
    # with the A operand streamed from LDS as in the MLP layers
    probe = dict(mfma_registers=dinr.probe_mfma(0, 20000), mfma_lds_operand=dinr.probe_mfma(1, 20000))
    log(f"measured BF16 MFMA rate (TFLOP/s): {probe}")
    roof["measured_peak_tflops"] = probe
    roof["frac_of_measured_peak"] = roof["achieved"] / max(probe.values())
    roof["traffic"] = traffic_from_profile(dom)
    # the weight-gradient kernels, bound by HBM: the stash bytes they read per
    # step over their HIP-event time
    if "wgrad" in kern:
        wb = wgrad_stash_bytes(spec, P_pts)
        wr = wb / (kern["wgrad"]["ms_per_step"] * 1e-3)
        roof["wgrad_hbm"] = dict(bound="hbm", achieved=wr / 1e9, peak=PEAK_HBM / 1e9,
                                 unit="GB/s", frac=wr / PEAK_HBM, bytes_per_step=wb,
                                 launches_per_step=kern["wgrad"]["launches_per_step"])
    loads = tuple(float(x) for x in args.serving_loads.split(","))
    serve = None if args.no_serving else serving(batch, trained, n_req=args.serving_requests,
                                                 rates=loads)
    paper = None if args.no_paper_net else paper_network(max(2, args.steps // 2), 1, ws)
    paper_d2 = None if args.no_paper_net else paper_network(2, 1, ws, sub=2, jitter=1)
    volume = None if args.no_volume else inference_volume(batch, trained)
    cone = None if args.no_c3 else cone_ragged(max(2, args.steps // 4), 1, ws)
    cpu, vs_oracle = None, None
    if not args.no_cpu:
        cpu, ref = cpu_baseline(batch)
        vs_oracle = errors_vs_oracle(batch, ref, 1024, 4 << 30)
        log(f"errors vs the FP64 oracle on {vs_oracle['rays']} rays: {json.dumps(vs_oracle)}")
    out = {
        "metric": "ray-samples/s fwd+bwd (one training step incl. Adam), BF16 matrix cores; "
                  "p50/p99 query ms",
        "value": P_pts / (ms_bf16 * 1e-3),
        "unit": "ray-samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_bf16,
        "step_ms_stats": STEP_STATS.get("c2"),
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
        "serving": serve,
        "paper_network": paper,
        "paper_network_2x2_random": paper_d2,
        "inference_volume": volume,
        "c3": cone,
        # latency at half the measured capacity
        "p50_ms": None if serve is None else serve["rates"][min(1, len(loads) - 1)]["p50_ms"],
        "p99_ms": None if serve is None else serve["rates"][min(1, len(loads) - 1)]["p99_ms"],
        "roofline": roof,
        "cpu_baseline": cpu,
        "vs_oracle_rel_err": vs_oracle,
        "status": status,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
