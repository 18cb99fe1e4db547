"""The forward projection that allocates nothing (dinr_forward_project_noalloc)
against dinr_forward_project, called through the C ABI: its scratch is the
library's static device array, so two calls in a row (the second smaller)
must each give exactly the projections and sample counts of the
workspace-based entry point, and a batch beyond the array is refused on the
host without touching the outputs."""
import numpy as np
import pytest

from paper_2404_19075_amd import dinr
from paper_2404_19075_amd import synth as S

from helpers import log, make_ctx, small_workload

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _noalloc(ctx):
    return ctx._lib.dinr_forward_project_noalloc


def _both(ctx, P, idx):
    R = idx.shape[0]
    p_ref = torch.full((R,), -7.0, device="cuda")
    n_ref = torch.full((R,), -7, dtype=torch.int32, device="cuda")
    ctx.forward_project(P, idx, proj=p_ref, n_out=n_ref)
    p_na = torch.full((R,), -7.0, device="cuda")
    n_na = torch.full((R,), -7, dtype=torch.int32, device="cuda")
    rc = _noalloc(ctx)(ctx._h, P.data_ptr(), idx.data_ptr(), R, p_na.data_ptr(),
                       n_na.data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert rc == dinr.OK, ctx._lib.dinr_last_error(ctx._h).decode()
    torch.cuda.synchronize()
    return (p_ref.cpu().numpy(), n_ref.cpu().numpy(), p_na.cpu().numpy(), n_na.cpu().numpy())


@pytest.mark.parametrize("name,R1,R2", [("c2", 65536, 3000), ("c3", 131072, 777)])
def test_noalloc_forward_matches_workspace_forward(name, R1, R2):
    w = S.workload(name)
    b = S.make_batch(w)
    log(f"noalloc forward {name}: R={R1} then R={R2}")
    # the smallest workspace a context accepts: the no-allocation entry point
    # does not use it
    ctx = make_ctx(w, b.B, dinr.BF16, ws_bytes=2 << 30)
    P = torch.tensor(b.params, device="cuda")
    for R in (R1, R2):
        idx = torch.tensor(b.idx[:R], device="cuda")
        p_ref, n_ref, p_na, n_na = _both(ctx, P, idx)
        log(f"  R={R}: points {int(n_ref.sum())}, equal proj {np.array_equal(p_ref, p_na)}, "
            f"equal n {np.array_equal(n_ref, n_na)}")
        assert np.array_equal(n_ref, n_na)
        assert np.array_equal(p_ref, p_na, equal_nan=True)
    ctx.close()


def test_noalloc_forward_refuses_a_batch_beyond_its_scratch():
    w = small_workload("c2", 1)
    b = S.make_batch(w)
    ctx = make_ctx(w, b.B, dinr.BF16, ws_bytes=64 << 20)
    P = torch.tensor(b.params, device="cuda")
    R = 1 << 20  # 64 MiB of ray records alone
    idx = torch.zeros(R, dtype=torch.int64, device="cuda")
    out = torch.full((R,), 3.0, device="cuda")
    rc = _noalloc(ctx)(ctx._h, P.data_ptr(), idx.data_ptr(), R, out.data_ptr(), None,
                       torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    msg = ctx._lib.dinr_last_error(ctx._h).decode()
    log(f"  refused: rc {rc}, '{msg}'")
    assert rc == dinr.ENOMEM and "static scratch" in msg
    assert bool(torch.all(out == 3.0))
    # the entry point still works after the refusal
    idx = torch.tensor(b.idx, device="cuda")
    p_ref, n_ref, p_na, n_na = _both(ctx, P, idx)
    assert np.array_equal(p_ref, p_na) and np.array_equal(n_ref, n_na)
    ctx.close()
