"""GPU path vs the FP64 oracle, element by element, on the same seeded inputs.

Tolerances (norm-wise relative error, ||x - x_ref|| / ||x_ref||):
  FP32 path: projections 1e-4, every gradient tensor 1e-3, loss 1e-4
  BF16 path: projections 2e-2; the whole gradient 5e-3, each tensor of the
             first layer (W1, b1) 5e-2, every other tensor 1.5e-2; loss 1e-3.
             The largest errors measured over these cases and the full-size
             ones are 2.6e-3 (whole gradient), 2.0e-2 (W1), 7.5e-3 (other
             tensors) and 8e-5 (loss).  The first layer's gradient sums
             products with high-frequency Fourier features that cancel
             heavily along a ray, so every rounding of the BF16 operands and
             every ReLU unit whose pre-activation rounds across zero is
             amplified there; the FP32 path shows the same 40-fold
             amplification of W1's error over the other tensors.
Sample counts are integers and must match exactly wherever the chord length
is not within 1e-4 (relative) of a multiple of the step; the oracle is then
re-run with the GPU's counts so that projections are compared on equal
quadratures.
"""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_2404_19075_amd import synth as S

from helpers import (check_grad, log, make_ctx, near_tie, rel, resolve_counts,
                     small_workload)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FP32, BF16 = 0, 1
TOL_PROJ = {FP32: 1e-4, BF16: 2e-2}
TOL_GRAD = {FP32: 1e-3, BF16: dict(first=5e-2, rest=1.5e-2, all=5e-3)}
TOL_LOSS = {FP32: 1e-4, BF16: 1e-3}


def run_forward(w, batch, prec, epoch=None):
    ctx = make_ctx(w, batch.B, prec)
    if epoch is not None:
        ctx.set_sample_epoch(epoch)
    P = torch.tensor(batch.params, device="cuda")
    idx = torch.tensor(batch.idx, device="cuda")
    n = torch.empty(len(batch.idx), dtype=torch.int32, device="cuda")
    proj = ctx.forward_project(P, idx, n_out=n)
    torch.cuda.synchronize()
    out = proj.cpu().numpy(), n.cpu().numpy()
    ctx.close()
    return out


def run_step(w, batch, prec, adam=None, recompute=False, epoch=None):
    ctx = make_ctx(w, batch.B, prec, recompute=recompute)
    if epoch is not None:
        ctx.set_sample_epoch(epoch)
    P = torch.tensor(batch.params, device="cuda")
    idx = torch.tensor(batch.idx, device="cuda")
    meas = torch.tensor(batch.meas, device="cuda")
    proj = torch.empty(len(batch.idx), dtype=torch.float32, device="cuda")
    grad, proj, loss, gnorm = ctx.step(P, idx, meas, proj=proj, adam=adam)
    torch.cuda.synchronize()
    out = dict(grad=grad.cpu().numpy(), proj=proj.cpu().numpy(), loss=float(loss.item()),
               gnorm=float(gnorm.item()), params=P.cpu().numpy(), status=ctx.step_status())
    ctx.close()
    return out


_ORACLE = {}


def oracle_step(key, w, b, n_override=None):
    """Oracle (loss, grad, proj), computed once per workload key."""
    if key not in _ORACLE:
        _ORACLE[key] = O.step(w.geom, w.mlp, w.sampling, b.B, b.params, b.idx, b.meas,
                              n_override=n_override)
    return _ORACLE[key]


@pytest.mark.parametrize("prec", [FP32, BF16])
def test_forward_c0(prec):
    b = S.make_batch("c0")
    w = b.workload
    log(f"test_forward_c0 prec={prec} R={len(b.idx)}")
    proj, n = run_forward(w, b, prec)
    ref, nref, _, _ = O.forward(w.geom, w.mlp, w.sampling, b.B, b.params, b.idx)
    assert np.array_equal(n, nref)
    e = rel(proj, ref)
    log(f"  proj rel err {e:.3e}")
    assert e <= TOL_PROJ[prec]


@pytest.mark.parametrize("prec", [FP32, BF16])
def test_step_c0(prec):
    b = S.make_batch("c0")
    w = b.workload
    log(f"test_step_c0 prec={prec}")
    out = run_step(w, b, prec)
    loss, grad, proj = oracle_step("c0", w, b)
    ep = rel(out["proj"], proj)
    el = abs(out["loss"] - loss) / loss
    log(f"  proj {ep:.3e} loss {el:.3e} (gpu {out['loss']:.6e} oracle {loss:.6e})")
    assert ep <= TOL_PROJ[prec]
    assert el <= TOL_LOSS[prec]
    check_grad(w, out["grad"], grad, TOL_GRAD[prec], f"c0 prec={prec}")
    gn = float(np.sum(out["grad"].astype(np.float64) ** 2))
    assert abs(out["gnorm"] - gn) <= 1e-9 * gn
    assert out["status"] == 0


@pytest.mark.parametrize("prec", [FP32, BF16])
def test_c1_network_ray_subset(prec):
    """The c1/c2 network (2C = 256, H = 256, L = 6) and geometry (256^2
    detector, 720 views, 256 samples per ray) on a ray subset the oracle
    finishes in seconds; 160 rays span many point tiles and a ragged last
    weight-gradient split."""
    w = small_workload("c1", 160)
    b = S.make_batch(w)
    log(f"test_c1_network_ray_subset prec={prec} R={len(b.idx)}")
    out = run_step(w, b, prec)
    loss, grad, proj = oracle_step("c1-160", w, b)
    ep = rel(out["proj"], proj)
    log(f"  proj {ep:.3e} loss gpu {out['loss']:.6e} oracle {loss:.6e}")
    assert ep <= TOL_PROJ[prec]
    check_grad(w, out["grad"], grad, TOL_GRAD[prec], f"c1 prec={prec}")


@pytest.mark.parametrize("prec", [FP32, BF16])
def test_cone_ragged_subset(prec):
    """c3 geometry and network (cone beam, n = clamp(ceil(l/h), 32, 512),
    L = 8) on 96 rays: rays span tile boundaries in the forward ray-sum."""
    w = small_workload("c3", 96)
    b = S.make_batch(w)
    log(f"test_cone_ragged_subset prec={prec}")
    proj_g, n_g = run_forward(w, b, prec)
    _, n_ref, _, ln = O.forward(w.geom, w.mlp, w.sampling, None, None, b.idx, field=(1, (0, 0, 0, 0, 0)))
    q = ln / w.sampling.h
    near_tie = np.abs(q - np.round(q)) < 1e-4 * np.maximum(q, 1)
    log(f"  n mismatches {int(np.sum(n_g != n_ref))}, near ties {int(near_tie.sum())}, "
        f"n range {n_g.min()}..{n_g.max()}")
    assert np.all((n_g == n_ref) | near_tie)
    ref, _, _, _ = O.forward(w.geom, w.mlp, w.sampling, b.B, b.params, b.idx, n_override=n_g)
    ep = rel(proj_g, ref)
    log(f"  proj rel err {ep:.3e}")
    assert ep <= TOL_PROJ[prec]
    out = run_step(w, b, prec)
    loss, grad, _ = O.step(w.geom, w.mlp, w.sampling, b.B, b.params, b.idx, b.meas, n_override=n_g)
    log(f"  loss gpu {out['loss']:.6e} oracle {loss:.6e}")
    check_grad(w, out["grad"], grad, TOL_GRAD[prec], f"c3 prec={prec}")


def test_adam_two_steps_c0():
    """Two training steps with Adam (Sec. II, App. C) on two c0 batches.  After
    each step the device's first and second moments equal the oracle's Adam
    recursion applied to the oracle's gradient (taken at the parameters the
    device started the step from), and the device's parameters moved by
    exactly the bias-corrected update of its own moments.  After the first
    step the parameters also equal the oracle's.  The second step exercises
    the moment decay and the bias correction beyond the first step."""
    from paper_2404_19075_amd import dinr
    w = S.workload("c0")
    b1_ = S.make_batch(w)
    b2_ = S.make_batch(w, seed_offset=1)
    lr, beta1, beta2, eps = 1e-3, 0.9, 0.999, 1e-8
    ctx = make_ctx(w, b1_.B, FP32)
    P = torch.tensor(b1_.params, device="cuda")
    m = torch.zeros(w.mlp.n_params, device="cuda")
    v = torch.zeros(w.mlp.n_params, device="cuda")
    p_dev = b1_.params.astype(np.float64)
    mo, vo = np.zeros_like(p_dev), np.zeros_like(p_dev)
    for k, bk in ((1, b1_), (2, b2_)):
        _, gk, _ = O.step(w.geom, w.mlp, w.sampling, bk.B, p_dev, bk.idx, bk.meas)
        po = p_dev.copy()
        O.adam(po, gk, mo, vo, lr, beta1, beta2, eps, k)
        ctx.step(P, torch.tensor(bk.idx, device="cuda"), torch.tensor(bk.meas, device="cuda"),
                 adam=(m, v, lr, beta1, beta2, eps, k))
        torch.cuda.synchronize()
        assert ctx.step_status() == dinr.OK
        pd, md, vd = (t.cpu().numpy().astype(np.float64) for t in (P, m, v))
        # m is linear and v quadratic in the gradient, whose FP32 error is a
        # few 1e-6 norm-wise on c0
        em, ev = rel(md, mo), rel(vd, vo)
        # the update of the device's own moments, in FP64
        upd = lr * (md / (1 - beta1 ** k)) / (np.sqrt(vd / (1 - beta2 ** k)) + eps)
        eu = np.abs((p_dev - upd) - pd).max()
        log(f"  step {k}: m rel {em:.2e} v rel {ev:.2e}, update vs own moments max abs {eu:.2e}")
        assert em <= 1e-4 and ev <= 1e-4
        assert eu <= 2e-8  # a few roundings of parameters of magnitude <= 1/8
        if k == 1:
            # a weight moves by ~lr sign(g): compare where |g| is not tiny
            mask = np.abs(gk) > 1e-6 * np.abs(gk).max()
            ep = np.abs(pd - po)[mask].max()
            log(f"  step 1 parameters vs the oracle: max abs {ep:.2e} on {mask.sum()}")
            assert ep <= 1e-6
        p_dev = pd
    ctx.close()


def test_edges_misses_bad_indices_and_small_batches():
    w = S.workload("c0")
    b = S.make_batch("c0")
    g = w.geom
    # pixel 0 of view 0 sits at |u| = |v| = 1.45 > 1: its ray misses the box
    idx = np.array([0, b.idx[0], g.n_proj + 5, -1, b.idx[1]], dtype=np.int64)
    bb = dataclasses.replace(b, idx=idx, meas=np.zeros(5, np.float32))
    proj, n = run_forward(w, bb, FP32)
    log(f"  edge proj {proj} n {n}")
    assert proj[0] == 0.0 and n[0] == 0
    assert np.isnan(proj[2]) and np.isnan(proj[3])
    ref, _, _, _ = O.forward(w.geom, w.mlp, w.sampling, b.B, b.params, idx[[1, 4]])
    assert rel(proj[[1, 4]], ref) <= 1e-4
    for R in (1, 3, 5):
        bb = dataclasses.replace(b, idx=b.idx[:R], meas=b.meas[:R])
        proj, _ = run_forward(w, bb, BF16)
        ref, _, _, _ = O.forward(w.geom, w.mlp, w.sampling, b.B, b.params, b.idx[:R])
        assert rel(proj, ref) <= 2e-2


def test_nonfinite_measurement_skips_adam():
    b = S.make_batch("c0")
    w = b.workload
    meas = b.meas.copy()
    meas[7] = np.nan
    bb = dataclasses.replace(b, meas=meas)
    m = torch.zeros(w.mlp.n_params, device="cuda")
    v = torch.zeros(w.mlp.n_params, device="cuda")
    out = run_step(w, bb, FP32, adam=(m, v, 1e-3, 0.9, 0.999, 1e-8, 1))
    assert out["status"] == -4
    assert np.array_equal(out["params"], b.params)


def test_run_to_run_bitwise_determinism():
    w = small_workload("c1", 160)
    b = S.make_batch(w)
    o1 = run_step(w, b, BF16)
    o2 = run_step(w, b, BF16)
    assert np.array_equal(o1["grad"], o2["grad"]) and np.array_equal(o1["proj"], o2["proj"])
    assert o1["loss"] == o2["loss"]


def test_batch_additivity_full_c1_size():
    """At the full c1 batch (65,536 rays x 256 samples), the gradient of the
    whole batch equals the size-weighted mean of the gradients of its halves
    (the averaging of Sec. II), and the projections of 48 sampled rays match
    the oracle one by one."""
    w = S.workload("c2")
    b = S.make_batch(w)
    log(f"full c1 size: R={len(b.idx)}")
    ctx = make_ctx(w, b.B, BF16, ws_bytes=64 << 30)
    P = torch.tensor(b.params, device="cuda")
    idx = torch.tensor(b.idx, device="cuda")
    meas = torch.tensor(b.meas, device="cuda")
    proj = torch.empty(len(b.idx), device="cuda")
    gfull, _, _, _ = ctx.step(P, idx, meas, proj=proj)
    h = len(b.idx) // 2
    # per-half gradients with the full-batch normalisation: dL/dpbar = 2 e / R
    g1 = ctx.project_backward(P, idx[:h].contiguous(),
                              (2.0 / len(b.idx)) * (proj[:h] - meas[:h]).contiguous())
    g2 = ctx.project_backward(P, idx[h:].contiguous(),
                              (2.0 / len(b.idx)) * (proj[h:] - meas[h:]).contiguous())
    torch.cuda.synchronize()
    gf = gfull.cpu().numpy().astype(np.float64)
    gs = (g1.cpu().numpy().astype(np.float64) + g2.cpu().numpy().astype(np.float64))
    e = rel(gs, gf)
    log(f"  additivity rel err {e:.3e}")
    assert e <= 1e-5
    rng = np.random.default_rng(0)
    pick = rng.choice(len(b.idx), 48, replace=False)
    ref, _, _, _ = O.forward(w.geom, w.mlp, w.sampling, b.B, b.params, b.idx[pick])
    ep = rel(proj.cpu().numpy()[pick], ref)
    log(f"  sampled proj rel err {ep:.3e}")
    assert ep <= 2e-2
    ctx.close()


def test_full_size_c3_ragged_cone():
    """The full c3 workload: 131,072 cone-beam rays with n = clamp(ceil(l/h),
    32, 512) samples, L = 8, BF16 with the forward recomputed in the
    backward, run as `dinr_step` runs it (two passes, several stash chunks).
    Every ray's sample count matches the oracle's chord, 48 sampled rays'
    projections match the oracle one by one, the loss is the FP64 mean of
    the GPU's own residuals, and the gradient of the batch equals the sum of
    the gradients of its halves."""
    w = S.workload("c3")
    b = S.make_batch(w)
    R = len(b.idx)
    log(f"full c3: R={R}")
    ctx = make_ctx(w, b.B, BF16, ws_bytes=64 << 30, recompute=True)
    P = torch.tensor(b.params, device="cuda")
    idx = torch.tensor(b.idx, device="cuda")
    meas = torch.tensor(b.meas, device="cuda")
    n = torch.empty(R, dtype=torch.int32, device="cuda")
    proj = ctx.forward_project(P, idx, n_out=n)
    proj2 = torch.empty(R, device="cuda")
    g, _, loss, _ = ctx.step(P, idx, meas, proj=proj2)
    torch.cuda.synchronize()
    assert ctx.step_status() == 0
    n_g = n.cpu().numpy()
    pg = proj.cpu().numpy()
    assert np.array_equal(pg, proj2.cpu().numpy())
    log(f"  points {int(n_g.sum())}, n range {n_g.min()}..{n_g.max()}")
    _, n_ref, _, ln = O.forward(w.geom, w.mlp, w.sampling, None, None, b.idx,
                                field=(1, (0, 0, 0, 0, 0)))
    q = ln / w.sampling.h
    near_tie = np.abs(q - np.round(q)) < 1e-4 * np.maximum(q, 1)
    assert np.all((n_g == n_ref) | near_tie)
    e64 = pg.astype(np.float64) - b.meas.astype(np.float64)
    lref = float(np.mean(e64 * e64))
    log(f"  loss gpu {loss.item():.9e} host {lref:.9e}")
    assert abs(loss.item() - lref) <= 1e-5 * lref
    rng = np.random.default_rng(3)
    pick = rng.choice(R, 48, replace=False)
    ref, _, _, _ = O.forward(w.geom, w.mlp, w.sampling, b.B, b.params, b.idx[pick],
                             n_override=n_g[pick])
    ep = rel(pg[pick], ref)
    log(f"  sampled proj rel err {ep:.3e}")
    assert ep <= TOL_PROJ[BF16]
    h = R // 2
    g1 = ctx.project_backward(P, idx[:h].contiguous(),
                              (2.0 / R) * (proj[:h] - meas[:h]).contiguous())
    g2 = ctx.project_backward(P, idx[h:].contiguous(),
                              (2.0 / R) * (proj[h:] - meas[h:]).contiguous())
    torch.cuda.synchronize()
    gs = g1.cpu().numpy().astype(np.float64) + g2.cpu().numpy().astype(np.float64)
    e = rel(gs, g.cpu().numpy().astype(np.float64))
    log(f"  additivity rel err {e:.3e}")
    assert e <= 1e-5
    ctx.close()


def test_full_size_paper_network_sampled():
    """The paper's network (Swish, five layers, linear output) on the full c2
    batch, 65,536 rays x 256 samples, BF16, as the benchmark's second leg runs
    it (one-pass step; a 64 GiB workspace forces several stash chunks).  The
    step's projections equal the forward kernel's, 48 sampled projections
    match the oracle one by one, the loss is the FP64 mean of the GPU's own
    residuals, and the gradient equals the sum of the two halves' gradients
    from the recomputing backward pass."""
    w = S.workload("paper")
    b = S.make_batch(w)
    R = len(b.idx)
    log(f"full paper network: R={R}")
    ctx = make_ctx(w, b.B, BF16, ws_bytes=64 << 30)
    P = torch.tensor(b.params, device="cuda")
    idx = torch.tensor(b.idx, device="cuda")
    meas = torch.tensor(b.meas, device="cuda")
    proj = ctx.forward_project(P, idx)
    proj2 = torch.empty(R, device="cuda")
    g, _, loss, _ = ctx.step(P, idx, meas, proj=proj2)
    torch.cuda.synchronize()
    assert ctx.step_status() == 0
    pg = proj.cpu().numpy()
    assert np.array_equal(pg, proj2.cpu().numpy())
    e64 = pg.astype(np.float64) - b.meas.astype(np.float64)
    lref = float(np.mean(e64 * e64))
    log(f"  loss gpu {loss.item():.9e} host {lref:.9e}")
    assert abs(loss.item() - lref) <= 1e-5 * lref
    pick = np.random.default_rng(5).choice(R, 48, replace=False)
    ref, _, _, _ = O.forward(w.geom, w.mlp, w.sampling, b.B, b.params, b.idx[pick])
    ep = rel(pg[pick], ref)
    log(f"  sampled proj rel err {ep:.3e}")
    assert ep <= TOL_PROJ[BF16]
    h = R // 2
    g1 = ctx.project_backward(P, idx[:h].contiguous(),
                              (2.0 / R) * (proj[:h] - meas[:h]).contiguous())
    g2 = ctx.project_backward(P, idx[h:].contiguous(),
                              (2.0 / R) * (proj[h:] - meas[h:]).contiguous())
    torch.cuda.synchronize()
    gs = g1.cpu().numpy().astype(np.float64) + g2.cpu().numpy().astype(np.float64)
    e = rel(gs, g.cpu().numpy().astype(np.float64))
    log(f"  additivity rel err {e:.3e}")
    assert e <= 1e-5
    ctx.close()


def test_full_size_paper_network_2x2_random_sampled():
    """The paper's sampling at full size: 65,536 projections x 2 x 2 rays x 256
    randomly placed samples on the Swish network (67 M samples, the two-pass
    step over several stash chunks).  48 sampled projections match the oracle
    at the same (seed, epoch), the loss is the FP64 mean of the GPU's own
    residuals, and the step's projections equal the forward's."""
    w0 = S.workload("paper")
    w = dataclasses.replace(w0, sampling=dataclasses.replace(w0.sampling, sub=2, jitter=1,
                                                             seed=31))
    b = S.make_batch(w)
    R = len(b.idx)
    ctx = make_ctx(w, b.B, BF16, ws_bytes=96 << 30)
    ctx.set_sample_epoch(12)
    P = torch.tensor(b.params, device="cuda")
    idx = torch.tensor(b.idx, device="cuda")
    meas = torch.tensor(b.meas, device="cuda")
    n = torch.empty(R, dtype=torch.int32, device="cuda")
    proj = ctx.forward_project(P, idx, n_out=n)
    proj2 = torch.empty(R, device="cuda")
    g, _, loss, _ = ctx.step(P, idx, meas, proj=proj2)
    torch.cuda.synchronize()
    assert ctx.step_status() == 0
    pg = proj.cpu().numpy()
    assert np.array_equal(pg, proj2.cpu().numpy())
    assert np.all(np.isfinite(g.cpu().numpy()))
    e64 = pg.astype(np.float64) - b.meas.astype(np.float64)
    lref = float(np.mean(e64 * e64))
    log(f"  loss gpu {loss.item():.9e} host {lref:.9e}")
    assert abs(loss.item() - lref) <= 1e-5 * lref
    pick = np.random.default_rng(9).choice(R, 48, replace=False)
    spe = dataclasses.replace(w.sampling, epoch=12)
    ref, n_ref, _, _ = O.forward(w.geom, w.mlp, spe, b.B, b.params, b.idx[pick])
    assert np.array_equal(n.cpu().numpy()[pick], n_ref.reshape(48, 4).sum(axis=1))
    ep = rel(pg[pick], ref)
    log(f"  sampled proj rel err {ep:.3e}")
    assert ep <= TOL_PROJ[BF16]
    ctx.close()


def test_autograd_function_matches_adjoint():
    from paper_2404_19075_amd import dinr
    w = S.workload("c0")
    b = S.make_batch("c0")
    ctx = make_ctx(w, b.B, FP32)
    P = torch.tensor(b.params, device="cuda", requires_grad=True)
    idx = torch.tensor(b.idx, device="cuda")
    meas = torch.tensor(b.meas, device="cuda")
    Fn = dinr.project_function()
    pbar = Fn.apply(P, idx, ctx)
    loss = torch.mean((meas - pbar) ** 2)
    loss.backward()
    grad, _, loss2, _ = ctx.step(P.detach(), idx, meas)
    torch.cuda.synchronize()
    assert rel(P.grad.cpu().numpy(), grad.cpu().numpy()) <= 1e-5
    assert abs(loss.item() - loss2.item()) <= 1e-6 * loss2.item()
    ctx.close()


@pytest.mark.parametrize("name,R", [("c0", 1024), ("c1", 160)])
def test_fused_pass_matches_recompute_pass(name, R):
    """The one-pass step (forward, loss and adjoint per tile of whole rays)
    and the two-pass step (forward kernel, loss kernel, backward kernel that
    recomputes the activations) evaluate the same arithmetic per point."""
    w = small_workload(name, R)
    b = S.make_batch(w)
    o1 = run_step(w, b, BF16)
    o2 = run_step(w, b, BF16, recompute=True)
    log(f"  {name}: proj equal {np.array_equal(o1['proj'], o2['proj'])}, "
        f"grad rel diff {rel(o1['grad'], o2['grad']):.3e}, loss {o1['loss']:.9e} {o2['loss']:.9e}")
    assert np.array_equal(o1["proj"], o2["proj"])
    assert rel(o1["grad"], o2["grad"]) <= 1e-6
    assert abs(o1["loss"] - o2["loss"]) <= 1e-12 * o2["loss"]


def swish_c0():
    """c0 with the paper's hidden activation and output (Swish, linear)."""
    w = S.workload("c0")
    return dataclasses.replace(w, mlp=dataclasses.replace(w.mlp, act=1, out_act=0))


@pytest.mark.parametrize("prec", [FP32, BF16])
def test_swish_c0_step(prec):
    """Swish hidden layers (Appendix B item 3) through the two-pass step: the
    forward kernel, then the backward kernel that stashes swish'(z) of every
    layer for the adjoint chain."""
    w = swish_c0()
    b = S.make_batch(w)
    log(f"test_swish_c0_step prec={prec}")
    proj_f, n = run_forward(w, b, prec)
    out = run_step(w, b, prec)
    loss, grad, proj = O.step(w.geom, w.mlp, w.sampling, b.B, b.params, b.idx, b.meas)
    ep, ef = rel(out["proj"], proj), rel(proj_f, proj)
    el = abs(out["loss"] - loss) / loss
    log(f"  proj {ep:.3e} forward {ef:.3e} loss {el:.3e}")
    assert ep <= TOL_PROJ[prec] and ef <= TOL_PROJ[prec]
    assert el <= TOL_LOSS[prec]
    check_grad(w, out["grad"], grad, TOL_GRAD[prec], f"swish c0 prec={prec}")
    assert out["status"] == 0


@pytest.mark.parametrize("prec", [FP32, BF16])
def test_paper_swish_network_ray_subset(prec):
    """The paper's network (2C = H = 256, five Swish layers, linear output,
    sigma_s = 0.5, sigma_t = 0.1) on 160 rays of the c2 geometry."""
    w = small_workload("paper", 160)
    b = S.make_batch(w)
    log(f"test_paper_swish_network_ray_subset prec={prec}")
    out = run_step(w, b, prec)
    loss, grad, proj = oracle_step("paper-160", w, b)
    ep = rel(out["proj"], proj)
    log(f"  proj {ep:.3e} loss gpu {out['loss']:.6e} oracle {loss:.6e}")
    assert ep <= TOL_PROJ[prec]
    check_grad(w, out["grad"], grad, TOL_GRAD[prec], f"paper prec={prec}")


def test_swish_fused_pass_matches_recompute_pass():
    """Swish network: the one-pass step and the two-pass step (forward kernel,
    loss, recomputing backward) evaluate the same arithmetic per point."""
    w = small_workload("paper", 160)
    b = S.make_batch(w)
    o1 = run_step(w, b, BF16)
    o2 = run_step(w, b, BF16, recompute=True)
    log(f"  grad rel diff {rel(o1['grad'], o2['grad']):.3e}")
    assert np.array_equal(o1["proj"], o2["proj"])
    assert rel(o1["grad"], o2["grad"]) <= 1e-6
    assert abs(o1["loss"] - o2["loss"]) <= 1e-12 * o2["loss"]


def with_sub(w, D, **samp):
    return dataclasses.replace(w, sampling=dataclasses.replace(w.sampling, sub=D, **samp))


@pytest.mark.parametrize("prec", [FP32, BF16])
def test_subpixel_rays_c0(prec):
    """D x D rays per projection (Appendix A, D = 2) on c0: every projection
    averages the samples of its 4 rays; the step takes the two-pass route."""
    w = with_sub(S.workload("c0"), 2)
    b = S.make_batch(w)
    log(f"test_subpixel_rays_c0 prec={prec}")
    proj_g, n_g = run_forward(w, b, prec)
    ref, n_ref, _, _ = O.forward(w.geom, w.mlp, w.sampling, b.B, b.params, b.idx)
    assert np.array_equal(n_g, n_ref.reshape(-1, 4).sum(axis=1))
    ep = rel(proj_g, ref)
    log(f"  forward proj rel err {ep:.3e}")
    assert ep <= TOL_PROJ[prec]
    out = run_step(w, b, prec)
    loss, grad, proj = O.step(w.geom, w.mlp, w.sampling, b.B, b.params, b.idx, b.meas)
    ep2, el = rel(out["proj"], proj), abs(out["loss"] - loss) / loss
    log(f"  step proj {ep2:.3e} loss {el:.3e}")
    assert ep2 <= TOL_PROJ[prec]
    assert el <= TOL_LOSS[prec]
    check_grad(w, out["grad"], grad, TOL_GRAD[prec], f"c0 D=2 prec={prec}")


@pytest.mark.parametrize("prec", [FP32, BF16])
def test_subpixel_rays_cone_variable_counts(prec):
    """Cone beam with n = clamp(ceil(l/h)) per ray and D = 2 (c3 geometry and
    network, 48 projections): |Phi| sums counts that differ between the rays
    of one projection, each sample weighted by its own ray's chord."""
    w = with_sub(small_workload("c3", 48), 2)
    b = S.make_batch(w)
    log(f"test_subpixel_rays_cone_variable_counts prec={prec}")
    proj_g, n_g = run_forward(w, b, prec)
    _, n_ref, _, ln = O.forward(w.geom, w.mlp, w.sampling, None, None, b.idx,
                                field=(1, (0, 0, 0, 0, 0)))
    q = ln / w.sampling.h
    tie = (np.abs(q - np.round(q)) < 1e-4 * np.maximum(q, 1)).reshape(-1, 4).any(axis=1)
    same = n_g == n_ref.reshape(-1, 4).sum(axis=1)
    log(f"  projections {len(n_g)}, count mismatches {int((~same).sum())}, near ties {int(tie.sum())}")
    assert np.all(same | tie)
    assert np.any(n_ref.reshape(-1, 4).min(axis=1) != n_ref.reshape(-1, 4).max(axis=1))
    # the oracle with per-ray counts that reproduce the device's totals
    n_ov = resolve_counts(n_g, n_ref, q, 4)
    ref, _, _, _ = O.forward(w.geom, w.mlp, w.sampling, b.B, b.params, b.idx, n_override=n_ov)
    ep = rel(proj_g, ref)
    log(f"  proj rel err {ep:.3e}")
    assert ep <= TOL_PROJ[prec]
    out = run_step(w, b, prec)
    loss, grad, _ = O.step(w.geom, w.mlp, w.sampling, b.B, b.params, b.idx, b.meas,
                           n_override=n_ov)
    el = abs(out["loss"] - loss) / loss
    log(f"  loss gpu {out['loss']:.6e} oracle {loss:.6e} ({el:.2e})")
    assert el <= TOL_LOSS[prec]
    check_grad(w, out["grad"], grad, TOL_GRAD[prec], f"c3 D=2 prec={prec}")


@pytest.mark.parametrize("prec", [FP32, BF16])
def test_random_sample_positions_c0(prec):
    """Stratified random positions (Sec. IV) drawn from Philox4x32-10 on both
    sides: forward, the one-pass step and the two-pass step match the oracle
    at the same (seed, epoch); another epoch moves the samples."""
    w0 = S.workload("c0")
    w = dataclasses.replace(w0, sampling=dataclasses.replace(w0.sampling, jitter=1, seed=2024))
    b = S.make_batch(w)
    spe = dataclasses.replace(w.sampling, epoch=5)
    log(f"test_random_sample_positions_c0 prec={prec}")
    proj_g, _ = run_forward(w, b, prec, epoch=5)
    ref, _, _, _ = O.forward(w.geom, w.mlp, spe, b.B, b.params, b.idx)
    mid, _, _, _ = O.forward(w.geom, w.mlp, w0.sampling, b.B, b.params, b.idx)
    ep = rel(proj_g, ref)
    log(f"  forward rel err {ep:.3e} (midpoints differ by {rel(mid, ref):.3e})")
    assert ep <= TOL_PROJ[prec]
    assert rel(mid, ref) > 10 * ep
    loss, grad, proj = O.step(w.geom, w.mlp, spe, b.B, b.params, b.idx, b.meas)
    for recompute in (False, True):
        out = run_step(w, b, prec, recompute=recompute, epoch=5)
        ep2 = rel(out["proj"], proj)
        log(f"  step recompute={recompute}: proj {ep2:.3e} loss gpu {out['loss']:.6e} "
            f"oracle {loss:.6e}")
        assert ep2 <= TOL_PROJ[prec]
        check_grad(w, out["grad"], grad, TOL_GRAD[prec], f"jitter recompute={recompute}")
    p6, _ = run_forward(w, b, prec, epoch=6)
    p5, _ = run_forward(w, b, prec, epoch=5)
    assert np.array_equal(p5, proj_g) and not np.array_equal(p6, proj_g)


def test_random_positions_subpixel_cone_bf16():
    """Random positions with D = 2 and per-ray counts on the c3 cone beam:
    counts differ from the oracle's only at near ties, projections and the
    two-pass step's gradient match the oracle at the same (seed, epoch)."""
    w0 = small_workload("c3", 32)
    w = dataclasses.replace(w0, sampling=dataclasses.replace(w0.sampling, sub=2, jitter=1,
                                                             seed=99))
    b = S.make_batch(w)
    proj_g, n_g = run_forward(w, b, BF16, epoch=3)
    spe = dataclasses.replace(w.sampling, epoch=3)
    _, n_ref, _, ln = O.forward(w.geom, w.mlp, spe, None, None, b.idx, field=(1, (0, 0, 0, 0, 0)))
    q = ln / w.sampling.h
    same = n_g == n_ref.reshape(-1, 4).sum(axis=1)
    log(f"  count mismatches {int((~same).sum())}, near ties {int(near_tie(q).sum())}")
    n_ov = resolve_counts(n_g, n_ref, q, 4)
    ref, _, _, _ = O.forward(w.geom, w.mlp, spe, b.B, b.params, b.idx, n_override=n_ov)
    ep = rel(proj_g, ref)
    log(f"  proj rel err {ep:.3e}")
    assert ep <= TOL_PROJ[BF16]
    out = run_step(w, b, BF16, epoch=3)
    loss, grad, _ = O.step(w.geom, w.mlp, spe, b.B, b.params, b.idx, b.meas, n_override=n_ov)
    el = abs(out["loss"] - loss) / loss
    log(f"  loss gpu {out['loss']:.6e} oracle {loss:.6e} ({el:.2e})")
    assert el <= TOL_LOSS[BF16]
    check_grad(w, out["grad"], grad, TOL_GRAD[BF16], "c3 D=2 jitter")


def test_subpixel_edges_misses_bad_indices_and_ray_limit():
    """D = 2 (and the largest D, 8): a projection whose rays all miss the FOV
    is 0 with |Phi| = 0, out-of-range indices give NaN, single projections and
    tiny batches match the oracle, and R D^2 beyond 2^31 - 2 is refused on the
    host before anything runs on the device."""
    from paper_2404_19075_amd import dinr
    b = S.make_batch("c0")
    g = b.workload.geom
    for D in (2, 8):
        w = with_sub(b.workload, D)
        idx = np.array([0, b.idx[0], g.n_proj + 5, -1, b.idx[1]], dtype=np.int64)
        bb = dataclasses.replace(b, workload=w, idx=idx, meas=np.zeros(5, np.float32))
        proj, n = run_forward(w, bb, FP32)
        log(f"  D={D} edge proj {proj} n {n}")
        assert proj[0] == 0.0 and n[0] == 0
        assert np.isnan(proj[2]) and np.isnan(proj[3])
        ref, n_ref, _, _ = O.forward(w.geom, w.mlp, w.sampling, b.B, b.params, idx[[1, 4]])
        assert np.array_equal(n[[1, 4]], n_ref.reshape(2, -1).sum(axis=1))
        assert rel(proj[[1, 4]], ref) <= 1e-4
        for R in (1, 3):
            bb = dataclasses.replace(b, workload=w, idx=b.idx[:R], meas=b.meas[:R])
            proj, _ = run_forward(w, bb, BF16)
            ref, _, _, _ = O.forward(w.geom, w.mlp, w.sampling, b.B, b.params, b.idx[:R])
            assert rel(proj, ref) <= 2e-2
    w = with_sub(b.workload, 8)
    ctx = make_ctx(w, b.B, FP32)
    P = torch.tensor(b.params, device="cuda")
    idx = torch.tensor(b.idx[:4], device="cuda")
    out = torch.empty(4, device="cuda")
    R_big = (2**31 - 2) // 64 + 1  # R D^2 = 2^31 - 2 + (64 - ...) > limit
    rc = ctx._lib.dinr_forward_project(ctx._h, P.data_ptr(), idx.data_ptr(), R_big, out.data_ptr(),
                                       None, None)
    assert rc == dinr.EINVAL
    assert "exceeds" in ctx._lib.dinr_last_error(ctx._h).decode()
    ctx.close()


def paper_sampling(w, D=2, n=256, jitter=1, seed=31):
    return dataclasses.replace(w, sampling=dataclasses.replace(w.sampling, n=n, sub=D,
                                                               jitter=jitter, seed=seed))


def step_kinds(w, b, prec, recompute=False, epoch=None, ws_bytes=2 << 30):
    """run_step plus the launches of each MLP kernel class it made."""
    from paper_2404_19075_amd import dinr
    ctx = make_ctx(w, b.B, prec, ws_bytes=ws_bytes, recompute=recompute)
    if epoch is not None:
        ctx.set_sample_epoch(epoch)
    ctx.profile(True)
    P = torch.tensor(b.params, device="cuda")
    idx = torch.tensor(b.idx, device="cuda")
    meas = torch.tensor(b.meas, device="cuda")
    proj = torch.empty(len(b.idx), dtype=torch.float32, device="cuda")
    grad, proj, loss, _ = ctx.step(P, idx, meas, proj=proj)
    torch.cuda.synchronize()
    kinds = {k: ctx.profile_read(v)[1] for k, v in (("fwd", dinr.PROF_MLP_FWD),
                                                    ("bwd", dinr.PROF_MLP_BWD),
                                                    ("one_pass", dinr.PROF_MLP_FUSED))}
    out = dict(grad=grad.cpu().numpy(), proj=proj.cpu().numpy(), loss=float(loss.item()),
               status=ctx.step_status(), kinds=kinds)
    ctx.close()
    return out


@pytest.mark.parametrize("prec", [FP32, BF16])
def test_grouped_one_pass_step_paper_sampling(prec):
    """The paper's network with its sampling (App. A: 2 x 2 rays per projection;
    Sec. IV: random positions; 256 samples per ray) on 160 projections: the
    one-pass step over groups of tiles that hold one projection each (BF16:
    four tiles of one ray each; FP32: eight tiles, two per ray) gives the
    two-pass step's projections bit for bit and its gradient to rounding,
    and matches the oracle at the same (seed, epoch)."""
    w = paper_sampling(small_workload("paper", 160))
    b = S.make_batch(w)
    log(f"test_grouped_one_pass_step_paper_sampling prec={prec}")
    o1 = step_kinds(w, b, prec, epoch=7)
    o2 = step_kinds(w, b, prec, recompute=True, epoch=7)
    log(f"  kernels: one-pass step {o1['kinds']}, two-pass step {o2['kinds']}")
    # one launch per stash chunk
    assert o1["kinds"]["one_pass"] >= 1 and o1["kinds"]["fwd"] == 0 and o1["kinds"]["bwd"] == 0
    assert o2["kinds"]["one_pass"] == 0 and o2["kinds"]["bwd"] >= 1
    eg = rel(o1["grad"], o2["grad"])
    log(f"  one-pass vs two-pass: proj equal {np.array_equal(o1['proj'], o2['proj'])}, "
        f"grad rel diff {eg:.2e}, loss {o1['loss']:.12e} {o2['loss']:.12e}")
    assert np.array_equal(o1["proj"], o2["proj"])
    assert eg <= 1e-6
    assert abs(o1["loss"] - o2["loss"]) <= 1e-12 * o2["loss"]
    spe = dataclasses.replace(w.sampling, epoch=7)
    loss, grad, proj = O.step(w.geom, w.mlp, spe, b.B, b.params, b.idx, b.meas)
    ep, el = rel(o1["proj"], proj), abs(o1["loss"] - loss) / loss
    log(f"  vs oracle: proj {ep:.3e} loss {el:.3e}")
    assert ep <= TOL_PROJ[prec] and el <= TOL_LOSS[prec]
    check_grad(w, o1["grad"], grad, TOL_GRAD[prec], f"grouped paper prec={prec}")
    assert o1["status"] == 0


def test_grouped_one_pass_step_paper_sampling_chunked():
    """As above (BF16) in a 1 GiB workspace, which holds the per-workgroup
    derivative ring and half of the stash: the grouped one-pass step runs in
    two or more stash chunks, the weight-gradient partials of each chunk are
    folded into the running compensated sums before the next, and the result
    matches the single-chunk step (projections bit for bit, gradient to
    rounding) and the oracle."""
    w = paper_sampling(small_workload("paper", 160))
    b = S.make_batch(w)
    log("test_grouped_one_pass_step_paper_sampling_chunked")
    o1 = step_kinds(w, b, BF16, epoch=7)
    o2 = step_kinds(w, b, BF16, epoch=7, ws_bytes=1 << 30)
    log(f"  kernels: one chunk {o1['kinds']}, small workspace {o2['kinds']}")
    assert o1["kinds"]["one_pass"] == 1 and o1["kinds"]["bwd"] == 0
    assert o2["kinds"]["one_pass"] >= 2 and o2["kinds"]["bwd"] == 0
    eg = rel(o2["grad"], o1["grad"])
    log(f"  chunked vs one chunk: grad rel diff {eg:.2e}")
    assert np.array_equal(o1["proj"], o2["proj"])
    assert eg <= 1e-6
    assert abs(o1["loss"] - o2["loss"]) <= 1e-12 * o1["loss"]
    spe = dataclasses.replace(w.sampling, epoch=7)
    loss, grad, proj = O.step(w.geom, w.mlp, spe, b.B, b.params, b.idx, b.meas)
    assert rel(o2["proj"], proj) <= TOL_PROJ[BF16]
    check_grad(w, o2["grad"], grad, TOL_GRAD[BF16], "grouped paper chunked")
    assert o2["status"] == 0


def test_grouped_one_pass_step_edges():
    """The grouped one-pass step (Swish c0 network, 2 x 2 rays of 256 samples,
    FP32: groups of eight 128-point tiles) on projections whose sub-rays
    partly miss the field of view (their rays padded with points of weight
    0), one that misses entirely (prediction 0) and an out-of-range index
    (NaN): the projections equal the two-pass step's and the oracle's, the
    loss is not finite and Adam is skipped; without the bad index the
    gradient matches the two-pass step's and the oracle's."""
    w0 = swish_c0()
    w = paper_sampling(w0, n=256, jitter=0)
    b = S.make_batch(w, n_rays=24)
    g = w.geom
    # view 0, row 16: col 0 lies at u = -1.45, outside the box, so its whole
    # pixel misses; col 5 lies at u = -0.98: of its sub-rays at u = -1.01 and
    # -0.96 one pair misses
    edge = np.array([16 * g.cols + 5, 16 * g.cols + 0], dtype=np.int64)
    idx = np.concatenate([edge, b.idx]).astype(np.int64)
    meas = np.concatenate([[0.3, 0.2], b.meas]).astype(np.float32)
    bb = dataclasses.replace(b, idx=idx, meas=meas)
    _, n_ref, _, _ = O.forward(w.geom, w.mlp, w.sampling, None, None, idx[:2],
                               field=(1, (0, 0, 0, 0, 0)))
    log(f"  edge sub-ray counts {n_ref.reshape(2, 4).tolist()}")
    assert n_ref[:4].min() == 0 and n_ref[:4].max() > 0 and n_ref[4:].max() == 0
    o1 = step_kinds(w, bb, FP32)
    o2 = step_kinds(w, bb, FP32, recompute=True)
    assert o1["kinds"]["one_pass"] >= 1 and o1["kinds"]["bwd"] == 0
    assert np.array_equal(o1["proj"], o2["proj"]) and o1["proj"][1] == 0.0
    assert rel(o1["grad"], o2["grad"]) <= 1e-6
    loss, grad, proj = O.step(w.geom, w.mlp, w.sampling, b.B, b.params, idx, meas)
    assert rel(o1["proj"], proj) <= TOL_PROJ[FP32]
    check_grad(w, o1["grad"], grad, TOL_GRAD[FP32], "grouped edges")
    # an out-of-range index: NaN prediction and loss, Adam skipped
    bad = dataclasses.replace(bb, idx=np.concatenate([[g.n_proj + 3], idx]).astype(np.int64),
                              meas=np.concatenate([[0.0], meas]).astype(np.float32))
    m = torch.zeros(w.mlp.n_params, device="cuda")
    v = torch.zeros(w.mlp.n_params, device="cuda")
    o3 = run_step(w, bad, FP32, adam=(m, v, 1e-3, 0.9, 0.999, 1e-8, 1))
    log(f"  bad index: proj[0] {o3['proj'][0]}, loss {o3['loss']}, status {o3['status']}")
    assert np.isnan(o3["proj"][0]) and not np.isfinite(o3["loss"])
    assert o3["status"] == -4 and np.array_equal(o3["params"], b.params)
    assert np.array_equal(o3["proj"][1:], o1["proj"])


def cylinder(w, radius=1.0, z0=-1.0, z1=1.0):
    """The workload in a cylindrical field of view (Sec. II, App. A): radius
    `radius` about the z axis, z in [z0, z1]; its bounds normalise x, y and z
    (App. B item 1)."""
    return dataclasses.replace(w, geom=dataclasses.replace(
        w.geom, fov_kind=1, fov=(radius, z0, z1, 0.0, 0.0, 0.0)))


@pytest.mark.parametrize("prec", [FP32, BF16])
@pytest.mark.parametrize("D", [1, 2])
def test_cylinder_fov_parallel_c0(prec, D):
    """c0 parallel beam in a cylindrical FOV of radius 1, z in [-1, 1]: counts
    (n or 0 per ray), projections and the step's loss and gradient match the
    oracle; at view 0 a pixel whose ray passes outside the radius and one
    whose ray passes above the z-slab give n = 0 and projection 0."""
    w = with_sub(cylinder(S.workload("c0")), D)
    b = S.make_batch(w)
    g = w.geom
    log(f"test_cylinder_fov_parallel_c0 prec={prec} D={D}")
    # view 0, row 16 (v = 0.047), col 0 (u = -1.45): outside the radius;
    # row 0 (v = -1.45), col 16 (u = 0.047): outside the z-slab
    radial, slab = 16 * g.cols + 0, 0 * g.cols + 16
    idx = np.concatenate([[radial, slab], b.idx]).astype(np.int64)
    bb = dataclasses.replace(b, idx=idx, meas=np.concatenate([[0.0, 0.0], b.meas]).astype(np.float32))
    proj_g, n_g = run_forward(w, bb, prec)
    ref, n_ref, _, ln = O.forward(w.geom, w.mlp, w.sampling, b.B, b.params, idx)
    assert n_g[0] == 0 and n_g[1] == 0 and proj_g[0] == 0.0 and proj_g[1] == 0.0
    assert np.array_equal(n_g, n_ref.reshape(len(idx), -1).sum(axis=1))
    assert np.any(ln.reshape(len(idx), -1)[2:] < 1.9)  # chords shorter than the box's
    ep = rel(proj_g, ref)
    log(f"  forward proj rel err {ep:.3e}")
    assert ep <= TOL_PROJ[prec]
    out = run_step(w, bb, prec)
    loss, grad, proj = O.step(w.geom, w.mlp, w.sampling, b.B, b.params, idx, bb.meas)
    ep2, el = rel(out["proj"], proj), abs(out["loss"] - loss) / loss
    log(f"  step proj {ep2:.3e} loss {el:.3e}")
    assert ep2 <= TOL_PROJ[prec] and el <= TOL_LOSS[prec]
    check_grad(w, out["grad"], grad, TOL_GRAD[prec], f"cylinder c0 D={D} prec={prec}")


@pytest.mark.parametrize("D", [1, 2])
def test_cylinder_fov_cone_per_ray_counts(D):
    """c3 cone beam (magnification 2) in a cylindrical FOV with per-ray counts
    n = clamp(ceil(l/h), 32, 512) from the cylinder chords, BF16: counts match
    the oracle except at near ties, projections and the two-pass step's
    gradient match it with the device's counts; rays missing through the
    radius and through the z-slab give 0."""
    w = with_sub(cylinder(small_workload("c3", 48)), D)
    b = S.make_batch(w)
    g = w.geom
    log(f"test_cylinder_fov_cone_per_ray_counts D={D}")
    # view 0: row 256 (v ~ 0), col 0 (u = -3.0, -1.5 at the axis): outside the
    # radius; row 0, col 256: outside the z-slab
    radial, slab = 256 * g.cols + 0, 0 * g.cols + 256
    idx = np.concatenate([[radial, slab], b.idx]).astype(np.int64)
    bb = dataclasses.replace(b, idx=idx, meas=np.concatenate([[0.0, 0.0], b.meas]).astype(np.float32))
    proj_g, n_g = run_forward(w, bb, BF16)
    _, n_ref, _, ln = O.forward(w.geom, w.mlp, w.sampling, None, None, idx,
                                field=(1, (0, 0, 0, 0, 0)))
    q = ln / w.sampling.h
    D2 = D * D
    assert n_g[0] == 0 and n_g[1] == 0 and proj_g[0] == 0.0 and proj_g[1] == 0.0
    nr = n_ref.reshape(len(idx), D2)
    log(f"  count range {nr[2:].min()}..{nr[2:].max()}, mismatches "
        f"{int(np.sum(n_g != nr.sum(axis=1)))}, near ties {int(near_tie(q).sum())}")
    hit = nr[2:][nr[2:] > 0]
    assert hit.min() >= 32 and hit.max() > 32
    n_ov = resolve_counts(n_g, n_ref, q, D2)
    ref, _, _, _ = O.forward(w.geom, w.mlp, w.sampling, b.B, b.params, idx, n_override=n_ov)
    ep = rel(proj_g, ref)
    log(f"  proj rel err {ep:.3e}")
    assert ep <= TOL_PROJ[BF16]
    out = run_step(w, bb, BF16)
    loss, grad, _ = O.step(w.geom, w.mlp, w.sampling, b.B, b.params, idx, bb.meas,
                           n_override=n_ov)
    el = abs(out["loss"] - loss) / loss
    log(f"  loss gpu {out['loss']:.6e} oracle {loss:.6e} ({el:.2e})")
    assert el <= TOL_LOSS[BF16]
    check_grad(w, out["grad"], grad, TOL_GRAD[BF16], f"cylinder cone D={D}")


def test_c1_network_ray_subset_chunked():
    """The c1 network on 160 rays with a workspace that holds a third of the
    stash: the step's adjoint runs in three chunks and still matches the
    oracle."""
    w = small_workload("c1", 160)
    b = S.make_batch(w)
    loss, grad, proj = oracle_step("c1-160", w, b)
    for prec in (FP32, BF16):
        ctx = make_ctx(w, b.B, prec, ws_bytes=(128 << 20) * (2 if prec == FP32 else 1))
        ctx.profile(True)
        P = torch.tensor(b.params, device="cuda")
        idx = torch.tensor(b.idx, device="cuda")
        meas = torch.tensor(b.meas, device="cuda")
        pr = torch.empty(len(b.idx), device="cuda")
        g, _, l_d, _ = ctx.step(P, idx, meas, proj=pr)
        torch.cuda.synchronize()
        # adjoint launches, one per chunk (one-pass BF16; the FP32 tile of 128
        # points cannot hold a 256-sample ray, so FP32 takes the two-pass step)
        chunks = max(ctx.profile_read(3)[1], ctx.profile_read(1)[1])
        ep = rel(pr.cpu().numpy(), proj)
        el = abs(l_d.item() - loss) / loss
        log(f"  prec={prec}: chunks {chunks}, proj {ep:.3e}, loss {el:.3e}")
        assert chunks == 3
        assert ep <= TOL_PROJ[prec] and el <= TOL_LOSS[prec]
        check_grad(w, g.cpu().numpy(), grad, TOL_GRAD[prec], f"c1 chunked prec={prec}")
        ctx.close()


@pytest.mark.parametrize("prec", [FP32, BF16])
def test_compensated_ray_sum_of_long_rays(prec):
    """Eq. (1)'s sum over many samples: four rays of 2^20 samples each (c0
    network).  A plain sequential FP32 sum of the oracle's own per-sample
    values misses the oracle's FP64 sum by far more than the device does: the
    kernel's ray-sum (a compensated scan within each 256-point tile, Kahan
    over the tiles) meets the oracle to within the rounding of the samples
    themselves."""
    w0 = S.workload("c0")
    w = dataclasses.replace(w0, sampling=dataclasses.replace(w0.sampling, n=1 << 20))
    b = S.make_batch(w, n_rays=4)
    proj_g, n_g = run_forward(w, b, prec)
    ref, n_ref, s_in, ln = O.forward(w.geom, w.mlp, w.sampling, b.B, b.params, b.idx)
    assert np.array_equal(n_g, n_ref)
    n = w.sampling.n
    naive_err, gpu_err = [], []
    for r, i in enumerate(b.idx):
        o, d, t = O.ray(w.geom, int(i))
        s = s_in[r] + (np.arange(n) + 0.5) * (ln[r] / n)
        pts = np.concatenate([o[None, :] + s[:, None] * d[None, :], np.full((n, 1), t)], axis=1)
        vals = O.field_points(w.geom, w.mlp, b.B, b.params, pts)  # mu0 M of every sample
        exact = float(np.sum(vals)) * (ln[r] / n)
        naive = float(np.cumsum(vals.astype(np.float32), dtype=np.float32)[-1]) * (ln[r] / n)
        naive_err.append(abs(naive - exact) / abs(exact))
        gpu_err.append(abs(float(proj_g[r]) - ref[r]) / abs(ref[r]))
        assert abs(exact - ref[r]) <= 1e-12 * abs(ref[r])
    log(f"  prec={prec}: sequential FP32 sum rel err {max(naive_err):.2e}, "
        f"device {max(gpu_err):.2e}")
    bound = 2e-6 if prec == FP32 else TOL_PROJ[BF16]
    assert max(gpu_err) <= bound
    if prec == FP32:
        assert min(naive_err) > 3 * bound


def test_training_on_c0_reduces_the_loss_tenfold():
    """Stochastic training as in Sec. II (a fresh batch of 1,024 projections
    each step, Adam lr 1e-3): the loss on a fixed held-out batch of the
    synthetic phantom falls at least tenfold within 400 steps (BF16)."""
    w = S.workload("c0")
    b = S.make_batch(w)
    ctx = make_ctx(w, b.B, BF16)
    P = torch.tensor(b.params, device="cuda")
    m, v = torch.zeros_like(P), torch.zeros_like(P)
    hold = S.make_batch(w, seed_offset=10_000)
    hidx = torch.tensor(hold.idx, device="cuda")
    hmeas = torch.tensor(hold.meas, device="cuda").double()

    def held_out_loss():
        p = ctx.forward_project(P, hidx)
        return float(torch.mean((p.double() - hmeas) ** 2).item())

    l0 = held_out_loss()
    for k in range(1, 401):
        bk = S.make_batch(w, seed_offset=k)
        ctx.step(P, torch.tensor(bk.idx, device="cuda"), torch.tensor(bk.meas, device="cuda"),
                 adam=(m, v, 1e-3, 0.9, 0.999, 1e-8, k))
    torch.cuda.synchronize()
    l1 = held_out_loss()
    log(f"  held-out loss {l0:.4e} -> {l1:.4e} ({l0 / l1:.1f}x)")
    assert ctx.step_status() == 0
    assert l1 * 10 <= l0
    ctx.close()
