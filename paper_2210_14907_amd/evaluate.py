"""Dense evaluation of a trained surrogate with the grid solution as fallback.

The surrogate u(x) = u^{sigma(x)}(x) is evaluated by `nbm_eval` on the
grid_n^d lattice x = -1 + 2 i / grid_n, streamed in tiles of consecutive
points (axis 0 fastest).  A judge solution given on the nodes of a coarser
grid (judge_n intervals; judge_n divides grid_n, so every judge node is a
lattice point) marks each tile: where the surrogate's largest error at the
judge nodes inside the tile exceeds the tolerance tau (or is not finite), the
tile falls back to the judge, and `nbm_grid_interp` writes the multilinear
interpolation of the judge solution at every point of that tile.  The error
after the fallback is measured on the values actually written.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class TileReport:
    tiles: int
    fallback_tiles: int
    linf: float            # surrogate error at the judge nodes (all tiles), before the fallback
    l2: float
    linf_after: float      # error of the written output at the judge nodes
    l2_after: float
    judge_points: int
    tau: float


def judge_mask_in_tile(grid_n: int, judge_n: int, d: int, tile: int, m: int):
    """Indices (within the tile) of lattice points that are judge nodes, and
    their flat judge-grid indices (judge grid has judge_n + 1 nodes per axis)."""
    stride = grid_n // judge_n
    q = np.arange(tile * m, (tile + 1) * m, dtype=np.int64)
    idx = np.stack([(q // grid_n ** a) % grid_n for a in range(d)], axis=1)
    on = np.all(idx % stride == 0, axis=1)
    j = idx[on] // stride
    flat = np.zeros(j.shape[0], dtype=np.int64)
    for a in range(d):
        flat += j[:, a] * (judge_n + 1) ** a
    return np.nonzero(on)[0], flat


def decide_fallback(tile_err: np.ndarray, tau: float) -> np.ndarray:
    """Per-tile fallback decision: error above tau, or not finite."""
    bad = ~np.isfinite(tile_err)
    return bad | (tile_err > tau)


def evaluate_lattice(nbm, params, grid_n: int, tile_points: int, judge_U=None, judge_n: int = 0,
                     tau: float = math.inf, out=None, keep=None):
    """Stream the lattice through the GPU.

    judge_U: nodal judge solution [(judge_n+1)^d] (numpy or device tensor,
    FP64).  out: optional device FP32 tensor [grid_n^d] that receives the
    final field (surrogate, or the interpolated judge on fallback tiles).
    keep: optional dict {tile: None} filled with host copies of those tiles.
    Returns a TileReport."""
    import torch

    d = nbm.wl.dim
    total = grid_n ** d
    if total % tile_points:
        raise ValueError("tile_points must divide grid_n^d")
    if judge_U is not None and (judge_n < 1 or grid_n % judge_n):
        raise ValueError("judge_n must divide grid_n")
    ntiles = total // tile_points
    dev = nbm.device
    buf = torch.empty(tile_points, dtype=torch.float32, device=dev)
    Ud = None
    if judge_U is not None:
        Ud = judge_U if torch.is_tensor(judge_U) else torch.tensor(np.ascontiguousarray(judge_U), device=dev)
        Ud = Ud.to(device=dev, dtype=torch.float64).contiguous()
    errs = np.zeros(ntiles)
    errs_after = np.zeros(ntiles)
    sq = sq_after = 0.0
    cnt = nfb = 0
    for t in range(ntiles):
        u = buf if out is None else out[t * tile_points:(t + 1) * tile_points]
        nbm.eval(params, None, m=tile_points, tile_index=t, grid_n=grid_n, out=u)
        if Ud is not None:
            loc, flat = judge_mask_in_tile(grid_n, judge_n, d, t, tile_points)
            loc_d = torch.from_numpy(loc).to(dev)
            ref = Ud[torch.from_numpy(flat).to(dev)]
            e = (u[loc_d].double() - ref).abs()
            e_max = float(e.max().item()) if e.numel() else 0.0
            errs[t] = e_max if math.isfinite(e_max) else math.inf
            sq += float((e * e).sum().item())
            cnt += int(e.numel())
            if decide_fallback(np.array([errs[t]]), tau)[0]:
                nbm.grid_interp(Ud, judge_n, t, grid_n, tile_points, out=u)
                nfb += 1
                e = (u[loc_d].double() - ref).abs()
                errs_after[t] = float(e.max().item()) if e.numel() else 0.0
            else:
                errs_after[t] = errs[t]
            sq_after += float((e * e).sum().item())
        if keep is not None and t in keep:
            keep[t] = u.cpu().numpy().copy()
    torch.cuda.synchronize()
    if Ud is None:
        return TileReport(ntiles, 0, float("nan"), float("nan"), float("nan"), float("nan"), 0, tau)
    c = max(cnt, 1)
    return TileReport(ntiles, nfb, float(errs.max()), math.sqrt(sq / c), float(errs_after.max()),
                      math.sqrt(sq_after / c), cnt, tau)
