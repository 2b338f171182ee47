"""FP64 two-network MLP for the oracle: plain point evaluation and a
hand-written reverse mode.

Paper Sec. 3: two networks u^- and u^+ represent the solution on each side of
Gamma; Sec. 4.1: sine-activated fully connected networks.  Each network has L
hidden layers of width W (L-1 hidden->hidden matrices, pinned by the 982
parameter count of Sec. 4.1 for L = 5, W = 10, d = 3), activation tanh or sin,
and a linear scalar output.  Parameter packing: net^- then net^+; per net
W1[W][d], b1, (W_l[W][W], b_l) for l = 2..L, w_out[W], b_out.
"""
from __future__ import annotations

import numpy as np

import nbm_inputs as I


def unpack(wl: I.Workload, theta: np.ndarray):
    """List of two nets; each net = [(W, b) per layer] + [(w_out[1, W], b_out[1])]."""
    W, d, L = wl.width, wl.dim, wl.depth
    nets = []
    off = 0
    for _ in range(2):
        layers = []
        shapes = [(W, d)] + [(W, W)] * (L - 1) + [(1, W)]
        for (fo, fi) in shapes:
            Wm = theta[off:off + fo * fi].reshape(fo, fi)
            off += fo * fi
            b = theta[off:off + fo]
            off += fo
            layers.append((Wm, b))
        nets.append(layers)
    assert off == theta.size
    return nets


def _act(wl, z):
    return np.tanh(z) if wl.act == I.ACT_TANH else np.sin(z)


def _dact(wl, z, a):
    return 1.0 - a * a if wl.act == I.ACT_TANH else np.cos(z)


def forward(wl: I.Workload, net, X: np.ndarray, keep=False):
    """u(X) for one net; X[m, d]."""
    a = X
    cache = [a]
    for (Wm, b) in net[:-1]:
        z = a @ Wm.T + b
        a = _act(wl, z)
        if keep:
            cache.append((z, a))
    w_out, b_out = net[-1]
    u = a @ w_out[0] + b_out[0]
    return (u, cache) if keep else u


def backward(wl: I.Workload, net, cache, ubar: np.ndarray):
    """Gradient of sum(ubar * u) w.r.t. the net's parameters, same packing."""
    grads = []
    w_out, _ = net[-1]
    a_last = cache[-1][1] if len(cache) > 1 else cache[0]
    g_wout = (ubar[:, None] * a_last).sum(axis=0)[None, :]
    g_bout = np.array([ubar.sum()])
    abar = ubar[:, None] * w_out[0][None, :]
    layer_grads = []
    for li in range(len(net) - 2, -1, -1):
        z, a = cache[li + 1]
        zbar = abar * _dact(wl, z, a)
        a_prev = cache[li] if li == 0 else cache[li][1]
        Wm, _ = net[li]
        layer_grads.append((zbar.T @ a_prev, zbar.sum(axis=0)))
        abar = zbar @ Wm
    layer_grads.reverse()
    for gW, gb in layer_grads:
        grads += [gW.ravel(), gb]
    grads += [g_wout.ravel(), g_bout]
    return np.concatenate(grads)


def eval_two(wl: I.Workload, theta: np.ndarray, X: np.ndarray, side_minus: np.ndarray,
             chunk: int = 1 << 16):
    """u^{sigma(x)}(x) at points X with given sides (True = minus)."""
    nets = unpack(wl, theta)
    out = np.empty(X.shape[0])
    for s, mask in ((0, side_minus), (1, ~side_minus)):
        idx = np.nonzero(mask)[0]
        for k in range(0, idx.size, chunk):
            sel = idx[k:k + chunk]
            out[sel] = forward(wl, nets[s], X[sel])
    return out
