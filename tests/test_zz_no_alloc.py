"""The allocation-free entry point nbm_forward_residual_noalloc (static
per-GPU scratch, no workspace) against nbm_forward_residual with a
workspace: same loss, residual vector and gradient, on two calls in a row
(the second with a smaller batch, so the scratch holds the first call's
contents when the second starts), on the fused 64-wide path and the layered
16-wide path; batches beyond the scratch and the Fourier problem are
rejected before any launch."""
import numpy as np
import pytest

import nbm_inputs as I
from tests.gpu_common import parity_batch

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _both(m, wl, theta, pts, bpts):
    p = torch.tensor(theta, dtype=torch.float32, device=DEV)
    tp = torch.tensor(pts, dtype=torch.float32, device=DEV)
    tb = torch.tensor(bpts, dtype=torch.float32, device=DEV).reshape(-1, wl.dim)
    n = pts.shape[0] + bpts.shape[0]
    ref = m.forward_residual(p, tp, tb, want_residual=True, want_grad=True)
    loss = torch.full((1,), -1.0, dtype=torch.float64, device=DEV)
    res = torch.full((n,), -1.0, dtype=torch.float32, device=DEV)
    grad = torch.full((m.P,), -1.0, dtype=torch.float32, device=DEV)
    m.forward_residual_noalloc(p, tp, tb, loss, residual=res, grad=grad)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in ref], [t.cpu().numpy() for t in (loss, res, grad)]


@pytest.mark.parametrize("wl", [I.C2, I.C2.replace(prec=I.PREC_BF16), I.C1], ids=["c2", "c2_bf16", "c1"])
def test_noalloc_matches_workspace_entry_point(wl):
    from paper_2210_14907_amd import NBM
    theta = I.xavier_params(wl, 3).astype(np.float32)
    big = parity_batch(wl, 4096, 96, 512, 0.02, seed=3)
    small = parity_batch(wl, 700, 20, 90, 0.02, seed=4)
    m = NBM(wl, max_points=big[0].shape[0], max_boundary=big[1].shape[0], cut_capacity=big[0].shape[0])
    for tag, (pts, bpts) in (("first", big), ("second, smaller", small)):
        print(f"[noalloc] {wl.name} {tag}: {pts.shape[0]} + {bpts.shape[0]} points", flush=True)
        (L0, r0, g0), (L1, r1, g1) = _both(m, wl, theta, pts, bpts)
        assert np.isfinite(L0).all() and L0[0] > 0
        # the same kernels on the same inputs: identical results
        assert L1[0] == L0[0], (L1, L0)
        assert np.array_equal(r1, r0) and np.array_equal(g1, g0)


def test_noalloc_full_c2_batch_fits():
    """The 64-wide sphere workload's whole training batch runs in the scratch."""
    from paper_2210_14907_amd import NBM
    wl = I.C2
    m = NBM(wl)
    pts, bpts = m.sample_points(seed=1, step=3)
    P, B = pts.cpu().numpy(), bpts.cpu().numpy()
    theta = I.xavier_params(wl, 0).astype(np.float32)
    (L0, r0, g0), (L1, r1, g1) = _both(m, wl, theta, P, B)
    assert L1[0] == L0[0] and np.array_equal(r1, r0) and np.array_equal(g1, g0)


def test_noalloc_rejects_what_does_not_fit():
    from paper_2210_14907_amd import NBM
    from paper_2210_14907_amd.binding import NbmError
    # 128-wide networks: the two-pass backward's tile buffers exceed the scratch
    wl = I.C3
    m = NBM(wl, max_points=2048, max_boundary=24)
    p = torch.tensor(I.xavier_params(wl, 0), dtype=torch.float32, device=DEV)
    pts, bpts = parity_batch(wl, 2048, 24, 0, 0.0)
    loss = torch.full((1,), 7.0, dtype=torch.float64, device=DEV)
    with pytest.raises(NbmError, match="scratch"):
        m.forward_residual_noalloc(p, torch.tensor(pts, dtype=torch.float32, device=DEV),
                                   torch.tensor(bpts, dtype=torch.float32, device=DEV), loss)
    torch.cuda.synchronize()
    assert loss.item() == 7.0   # nothing was launched
    # the Fourier problem's tables live in a prepared workspace
    wl4 = I.C4
    m4 = NBM(wl4, max_points=256, max_boundary=4)
    p4 = torch.tensor(I.xavier_params(wl4, 0), dtype=torch.float32, device=DEV)
    q, qb = parity_batch(wl4, 256, 4, 0, 0.0)
    with pytest.raises(NbmError, match="Fourier"):
        m4.forward_residual_noalloc(p4, torch.tensor(q, dtype=torch.float32, device=DEV),
                                    torch.tensor(qb, dtype=torch.float32, device=DEV), loss)
