"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol declared in include/nbm.h, validates configurations and sizes
workspaces."""
import ctypes
import re
from pathlib import Path

import pytest

import nbm_inputs as I

ROOT = Path(__file__).resolve().parents[1]


def _decls():
    txt = (ROOT / "include" / "nbm.h").read_text()
    return sorted(set(re.findall(r"\b(nbm_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_2210_14907_amd import binding as B
    L = B.lib()
    names = _decls()
    assert len(names) >= 11
    for nme in names:
        assert hasattr(L, nme), nme
    assert set(B.EXPORTS) == set(names)


def _cfg(wl, **over):
    from paper_2210_14907_amd import binding as B
    c = B.NbmConfig()
    c.dim, c.width, c.depth, c.act, c.prec, c.h = wl.dim, wl.width, wl.depth, wl.act, wl.prec, wl.h
    c.interface_kind, c.radius, c.star_amp = wl.interface, wl.radius, wl.star_amp
    c.mu_minus, c.mu_plus, c.problem = wl.mu_minus, wl.mu_plus, wl.problem
    c.max_points, c.max_boundary = wl.n_points, wl.n_boundary
    for k, v in over.items():
        setattr(c, k, v)
    return c


def _create(c):
    from paper_2210_14907_amd import binding as B
    h = ctypes.c_void_p()
    rc = B.lib().nbm_create(ctypes.byref(c), ctypes.byref(h))
    return rc, h


@pytest.mark.parametrize("wl", [I.C1, I.C2, I.C3], ids=["c1", "c2", "c3"])
def test_create_counts_and_workspace(wl):
    from paper_2210_14907_amd import binding as B
    rc, h = _create(_cfg(wl))
    assert rc == 0
    assert B.lib().nbm_param_count(h) == wl.n_params
    ws = B.lib().nbm_workspace_bytes(h, wl.n_points, wl.n_boundary)
    assert ws > 0
    # smaller batches need no more; past the capacity the query is rejected
    assert 0 < B.lib().nbm_workspace_bytes(h, wl.n_points // 4, 0) < ws
    assert B.lib().nbm_workspace_bytes(h, wl.n_points + 1, 0) == 0
    assert B.lib().nbm_workspace_bytes(h, 1, wl.n_boundary + 1) == 0
    assert B.lib().nbm_workspace_bytes(h, -1, 0) == 0
    B.lib().nbm_destroy(h)


def test_create_rejects_bad_configs():
    from paper_2210_14907_amd import binding as B
    bad = [dict(dim=4), dict(depth=1), dict(h=0.3), dict(h=0.01), dict(mu_minus=0.0),
           dict(k_minus=-1.0), dict(k_plus=float("nan")), dict(width=24), dict(act=7), dict(max_points=0),
           dict(levels=7), dict(levels=-1), dict(h=2.0 ** -18, levels=3)]
    for over in bad:
        rc, _ = _create(_cfg(I.C2, **over))
        assert rc < 0, over
        assert len(B.lib().nbm_last_error()) > 0
    rc, _ = _create(_cfg(I.C2, width=16, prec=I.PREC_BF16))
    assert rc == -3   # BF16 needs W >= 64 (K chunk of 8 per lane group)
    rc, _ = _create(_cfg(I.C4))   # Fourier problem without a mode table
    assert rc == -1
