"""Host logic of the dense evaluation and grid fallback (no GPU): judge-node
selection inside lattice tiles and the forced fallback cases (tau = 0 makes
every tile fall back, tau = inf none, non-finite errors always)."""
import math

import numpy as np

from paper_2210_14907_amd.evaluate import decide_fallback, judge_mask_in_tile


def test_judge_nodes_inside_tiles_cover_judge_grid():
    grid_n, judge_n, d, m = 16, 4, 3, 256
    seen = []
    for t in range(grid_n ** d // m):
        loc, flat = judge_mask_in_tile(grid_n, judge_n, d, t, m)
        q = t * m + loc
        idx = np.stack([(q // grid_n ** a) % grid_n for a in range(d)], axis=1)
        assert np.all(idx % (grid_n // judge_n) == 0)
        seen.append(flat)
    seen = np.concatenate(seen)
    # every judge node with index < judge_n along each axis appears once
    assert len(seen) == judge_n ** d and len(np.unique(seen)) == judge_n ** d


def test_forced_fallback_cases():
    err = np.array([0.0, 1e-3, 0.5, np.nan, np.inf])
    assert decide_fallback(err, 0.0).tolist() == [False, True, True, True, True]
    assert decide_fallback(err, math.inf).tolist() == [False, False, False, True, True]
    assert decide_fallback(err, 0.1).tolist() == [False, False, True, True, True]
