"""Full-size launches: the star workload at its configured batch (1,048,576 +
3,072 points, h = 1/1024, two 3->128x4->1 sine nets, BF16 operands) and dense
evaluation tiles of 2^24 points of the 1024^3 lattice.  The oracle checks a
sample of outputs one by one (each point's residual depends only on that
point and the parameters); the loss is checked against the mean square of the
returned residual vector."""
import numpy as np
import pytest

import nbm_inputs as I
from oracle import geometry as G
from oracle import mlp as M
from oracle import nbm as N
from oracle import scheme as S
from tests.gpu_common import max_rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_c4_full_batch_sampled_parity():
    from paper_2210_14907_amd import NBM
    wl = I.C4
    print("[scale] c4 full batch", flush=True)
    nbm = NBM(wl)
    theta = I.xavier_params(wl, 0).astype(np.float32).astype(np.float64)
    p = torch.tensor(theta, dtype=torch.float32, device=nbm.device)
    pts, bpts = nbm.sample_points(seed=1, step=1)
    loss, res, grad = nbm.forward_residual(p, pts, bpts, want_residual=True, want_grad=True)
    torch.cuda.synchronize()
    r = res.cpu().numpy().astype(np.float64)
    L = loss.item()
    counts = nbm.batch_counts().cpu().numpy()
    print(f"[scale] c4 loss {L:.6e} classes {counts[:5].tolist()} overflow {counts[5]}", flush=True)
    assert counts[5] == 0 and counts[2] > 0
    assert np.isfinite(L) and np.all(np.isfinite(grad.cpu().numpy()))
    assert abs(L - np.mean(r * r)) <= 1e-5 * L
    # sampled per-point residuals against the oracle (all cut cells + random others)
    P = pts.cpu().numpy().astype(np.float64)
    B = bpts.cpu().numpy().astype(np.float64)
    cls, _ = S.classify(wl, P, wl.h)
    cut = np.nonzero(cls == S.CLASS_CUT)[0]
    rng = np.random.default_rng(0)
    idx = np.concatenate([cut[:300], rng.choice(P.shape[0], 700, replace=False)])
    bidx = rng.choice(B.shape[0], 200, replace=False)
    ro = N.residuals(wl, theta, P[idx], B[bidx])
    e_i = max_rel(r[idx], ro["r"])
    e_b = max_rel(r[P.shape[0] + bidx], ro["rb"])
    un = ro["cls"] != S.CLASS_CUT
    e_u = max_rel(r[idx][un], ro["r"][un])
    print(f"[scale] c4 sampled residual rel: interior {e_i:.2e} uncut {e_u:.2e} boundary {e_b:.2e}", flush=True)
    assert e_i <= 2e-2 and e_b <= 2e-2 and e_u <= 2e-2


def test_c5_eval_tiles_of_the_1024_lattice():
    from paper_2210_14907_amd import NBM
    wl = I.C4
    m = 1 << 24
    nbm = NBM(wl, max_points=m, max_boundary=0, eval_only=True)
    theta = I.xavier_params(wl, 1).astype(np.float32).astype(np.float64)
    p = torch.tensor(theta, dtype=torch.float32, device=nbm.device)
    gn = 1024
    rng = np.random.default_rng(3)
    for tile in (0, 31, 63):
        u = nbm.eval(p, None, m=m, tile_index=tile, grid_n=gn).cpu().numpy()
        loc = rng.choice(m, 2000, replace=False)
        q = tile * m + loc
        x = np.stack([(q // gn ** a) % gn for a in range(3)], axis=1) * (2.0 / gn) - 1.0
        ref = M.eval_two(wl, theta, x, G.side_minus(wl, x))
        tie = np.abs(G.phi(wl, x)) < 1e-12
        e = max_rel(u[loc][~tie], ref[~tie])
        print(f"[scale] c5 tile {tile}: sampled rel {e:.2e}", flush=True)
        assert e <= 2e-2
