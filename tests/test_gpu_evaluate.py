"""Dense evaluation with the grid fallback, on the GPU through the C ABI:
tiles whose surrogate error at the judge nodes exceeds tau get the judge's
multilinear interpolation written at every point (nbm_grid_interp), checked
against the oracle's interpolation; tau = 0 forces every tile to fall back,
tau = inf none, and a middle tau splits the tiles."""
import math

import numpy as np
import pytest

import nbm_inputs as I
from oracle import geometry as G
from oracle import grid as OG
from oracle import mlp as M

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _lattice(grid_n, d, lo, hi):
    q = np.arange(lo, hi, dtype=np.int64)
    return np.stack([(q // grid_n ** a) % grid_n for a in range(d)], axis=1) * (2.0 / grid_n) - 1.0


def test_grid_fallback_tiles_take_the_interpolated_judge():
    from paper_2210_14907_amd import NBM
    from paper_2210_14907_amd.evaluate import evaluate_lattice
    wl = I.C2
    grid_n, judge_n, tile = 64, 16, 64 ** 3 // 8
    gs = OG.GridSystem(wl, judge_n)
    U = gs.solve()
    theta = I.xavier_params(wl, 2).astype(np.float32).astype(np.float64)
    nbm = NBM(wl, max_points=tile, max_boundary=0, eval_only=True)
    p = torch.tensor(theta, dtype=torch.float32, device=nbm.device)
    x = _lattice(grid_n, 3, 0, grid_n ** 3)
    interp = OG.interp_grid(U, judge_n, 3, x)
    side = G.side_minus(wl, x)
    net = M.eval_two(wl, theta, x, side)
    tie = np.abs(G.phi(wl, x)) < 1e-12
    scale = np.abs(interp).max()

    out = torch.empty(grid_n ** 3, dtype=torch.float32, device=nbm.device)
    rep = evaluate_lattice(nbm, p, grid_n, tile, judge_U=U, judge_n=judge_n, tau=0.0, out=out)
    o = out.cpu().numpy().astype(np.float64)
    print(f"[fallback] tau=0: {rep}", flush=True)
    assert rep.tiles == 8 and rep.fallback_tiles == 8 and rep.judge_points == judge_n ** 3
    assert np.abs(o - interp).max() <= 1e-6 * scale
    assert rep.linf > 0.0 and rep.linf_after <= 1e-6 * scale

    rep = evaluate_lattice(nbm, p, grid_n, tile, judge_U=U, judge_n=judge_n, tau=math.inf, out=out)
    o = out.cpu().numpy().astype(np.float64)
    print(f"[fallback] tau=inf: {rep}", flush=True)
    assert rep.fallback_tiles == 0 and rep.linf_after == rep.linf
    assert np.abs(o - net)[~tie].max() <= 1e-5 * np.abs(net).max()

    # a middle tolerance: per tile, the output is either all surrogate or all judge
    from paper_2210_14907_amd.evaluate import judge_mask_in_tile
    errs = []
    sl = [slice(t * tile, (t + 1) * tile) for t in range(8)]
    for t in range(8):
        loc, flat = judge_mask_in_tile(grid_n, judge_n, 3, t, tile)
        errs.append(np.abs(net[sl[t]][loc] - U[flat]).max())
    tau = float(np.median(errs))
    rep = evaluate_lattice(nbm, p, grid_n, tile, judge_U=U, judge_n=judge_n, tau=tau, out=out)
    o = out.cpu().numpy().astype(np.float64)
    fb = [e > tau for e in errs]
    print(f"[fallback] tau={tau:.3e}: {rep}; tiles falling back {fb}", flush=True)
    assert rep.fallback_tiles == sum(fb) and 0 < sum(fb) < 8
    for t in range(8):
        ref = interp[sl[t]] if fb[t] else net[sl[t]]
        ok = np.ones(tile, dtype=bool) if fb[t] else ~tie[sl[t]]
        assert np.abs(o[sl[t]] - ref)[ok].max() <= 1e-5 * max(scale, np.abs(net).max()), t
    assert rep.linf_after <= tau + 1e-6 * scale
