"""Dense evaluation of a trained surrogate and the grid fallback.

The surrogate u(x) = u^{sigma(x)}(x) is evaluated by `nbm_eval` on the
grid_n^d lattice x = -1 + 2 i / grid_n, streamed in tiles of consecutive
points (axis 0 fastest).  A judge solution given on the nodes of a coarser
grid (judge_n intervals; judge_n divides grid_n) marks each tile: where the
surrogate's largest error at the judge nodes inside the tile exceeds the
tolerance tau, the tile falls back to the judge's multilinear interpolation.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class TileReport:
    tiles: int
    fallback_tiles: int
    linf: float            # surrogate error at judge nodes (all tiles)
    l2: float
    linf_after: float      # error after fallback
    judge_points: int


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
                     tau: float = math.inf, keep=None):
    """Stream the lattice through the GPU; returns a TileReport (and fills
    keep[tile] = u for tiles listed in the dict `keep`)."""
    import torch

    d = nbm.wl.dim
    total = grid_n ** d
    if total % tile_points:
        raise ValueError("tile_points must divide grid_n^d")
    ntiles = total // tile_points
    out = torch.empty(tile_points, dtype=torch.float32, device=nbm.device)
    errs = np.zeros(ntiles)
    sq = 0.0
    cnt = 0
    for t in range(ntiles):
        nbm.eval(params, None, m=tile_points, tile_index=t, grid_n=grid_n, out=out)
        if judge_U is None and keep is None:
            continue
        u = out.cpu().numpy()
        if keep is not None and t in keep:
            keep[t] = u.copy()
        if judge_U is not None:
            loc, flat = judge_mask_in_tile(grid_n, judge_n, d, t, tile_points)
            e = np.abs(u[loc].astype(np.float64) - judge_U[flat])
            errs[t] = e.max() if e.size else 0.0
            sq += float((e * e).sum())
            cnt += e.size
    torch.cuda.synchronize()
    if judge_U is None:
        return TileReport(ntiles, 0, float("nan"), float("nan"), float("nan"), 0)
    fb = decide_fallback(errs, tau)
    after = np.where(fb, 0.0, errs)   # fallback tiles take the judge values at its nodes
    return TileReport(ntiles, int(fb.sum()), float(errs.max()), math.sqrt(sq / max(cnt, 1)),
                      float(after.max()), cnt)
