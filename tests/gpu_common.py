"""Helpers shared by the GPU parity tests: seeded inputs and oracle calls."""
import math

import numpy as np

import nbm_inputs as I
from oracle import geometry as G


def near_star_points(wl, n, band, seed=9):
    """Lattice points within `band` (radially) of the star interface: the star
    radius in direction v is R + amp sin(5 theta) sin(4 psi), read off the
    oracle level set along the ray."""
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    # phi(t v) = t - R(v) on a ray, so R(v) = t - phi(t v) for any t > 0
    Rv = 0.5 - G.phi(wl, 0.5 * v)
    r = Rv + 0.5 + rng.uniform(-band, band, size=n) - 0.5
    x = v * r[:, None]
    q = float(2 ** 22)
    return np.round(x * q) / q


def parity_batch(wl, n, nb, n_near, band, seed=1):
    pts, bpts = I.collocation_batch(wl, n, nb, seed=seed)
    if n_near:
        star = wl.interface == I.IFACE_STAR or (wl.interface == I.IFACE_GRID and wl.phi_shape == I.IFACE_STAR)
        if star:
            near = near_star_points(wl, n_near, band, seed=seed + 11)
        else:
            near = I.near_interface_points(wl, n_near, band, seed=seed + 11)
        lo, hi = -1 + wl.h, 1 - wl.h
        near = np.clip(near, lo, hi)
        pts = np.concatenate([pts, near])
    return pts, bpts


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (den if den > 0 else 1.0)


def max_rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max()
    return np.abs(a - b).max() / (den if den > 0 else 1.0)


def param_blocks(wl):
    """(name, slice) of every parameter block of both nets, in packing order:
    W1, b1, (W_l, b_l) for l = 2..L, w_out, b_out per net."""
    W, d, L = wl.width, wl.dim, wl.depth
    out, off = [], 0
    for net in ("minus", "plus"):
        shapes = [("W1", W * d), ("b1", W)]
        for l in range(2, L + 1):
            shapes += [(f"W{l}", W * W), (f"b{l}", W)]
        shapes += [("wout", W), ("bout", 1)]
        for name, size in shapes:
            out.append((f"{net}.{name}", slice(off, off + size)))
            off += size
    assert off == wl.n_params
    return out


def grad_block_ratios(wl, g, g_o, tol, floor=1e-3, scale=None):
    """Per parameter block, the largest |g - g_o| / (tol (|g_o| + floor max|g_o|_block)):
    every entry of every block must be within tol of the oracle relative to its
    own size, entries far below the block's largest one relative to that.
    When the gradient is a sum of parts (resolution levels), scale holds the
    sum of the parts' magnitudes and the floor is taken relative to it: the
    parts' rounding does not cancel where their values do."""
    g = np.asarray(g, dtype=np.float64)
    g_o = np.asarray(g_o, dtype=np.float64)
    sc = np.abs(g_o) if scale is None else np.asarray(scale, dtype=np.float64)
    out = {}
    for name, sl in param_blocks(wl):
        a, b = g[sl], g_o[sl]
        bound = tol * (np.abs(b) + floor * sc[sl].max())
        out[name] = float(np.max(np.abs(a - b) / np.where(bound > 0, bound, 1.0)))
    return out
