"""NBM training step, plain definition (oracle, FP64).

Paper Sec. 3: the networks are evaluated at the vertices of an implicit cell
placed at each random collocation point, each point contributes the locally
preconditioned residual r_p of the bootstrapped discretisation, the residual
contributions are aggregated into a global loss, automatic differentiation
passes across the kernels, and Adam adjusts the parameters.  The loss equation
itself is missing from the text; the reading used here is the mean of the
squared point residuals over the interior and boundary points,

    L = (sum_p r_p^2 + sum_b r_b^2) / (N + N_b),

with r_p from `scheme` and r_b = (2d/h^2)(U(x_b) - g(x_b)).  U at a node is
the value of the network of the node's own side, evaluated at the node in
FP64 (point evaluation); stencil differences are formed from those values.
With a coefficient contrast the lagged low-mu normal derivative in the jump
extension is the central difference (step h) of the low-mu network around the
node, treated as a constant (no gradient flows through it).
"""
from __future__ import annotations

import numpy as np

import nbm_inputs as I
from . import geometry as G
from . import mlp as M
from . import scheme as S
from .problems import Problem


def _eval_net(wl, net, X, chunk=1 << 15):
    out = np.empty(X.shape[0])
    for k in range(0, X.shape[0], chunk):
        out[k:k + chunk] = M.forward(wl, net, X[k:k + chunk])
    return out


def _grad_net(wl, net, X, ubar, chunk=1 << 15):
    g = None
    for k in range(0, X.shape[0], chunk):
        u, cache = M.forward(wl, net, X[k:k + chunk], keep=True)
        gk = M.backward(wl, net, cache, ubar[k:k + chunk])
        g = gk if g is None else g + gk
    if g is None:
        g = M.backward(wl, net, [np.zeros((0, X.shape[1]))] +
                       [(np.zeros((0, wl.width)), np.zeros((0, wl.width)))] * wl.depth,
                       np.zeros(0))
    return g


def network_provider(wl: I.Workload, theta: np.ndarray):
    """Value provider u(s, X): network of side s evaluated at X (FP64)."""
    nets = M.unpack(wl, theta)
    return lambda s, X: _eval_net(wl, nets[s], X)


def exact_provider(wl: I.Workload):
    """Value provider from the closed-form solution of a manufactured problem."""
    prob = Problem(wl)
    return lambda s, X: prob.u_side(s, X)


def residuals(wl: I.Workload, theta: np.ndarray, pts: np.ndarray, bpts: np.ndarray,
              h: float = None, provider=None, glo_override=None):
    """Point residuals, loss and the evaluation requests needed for the
    gradient.  Returns dict: r[n], rb[nb], cls[n], loss, and `req` = per side
    a list of (row ids, X, dr/dU) blocks for the reverse pass.

    provider(s, X) gives the side-s function at points X (default: the
    networks in theta).  glo_override[m_cut, 2d+1, d] replaces the lagged
    low-mu gradients at the cut-cell nodes (used to hold them fixed in
    finite-difference checks)."""
    h = wl.h if h is None else h
    prob = Problem(wl)
    nets = M.unpack(wl, theta) if theta is not None else None
    if provider is None:
        provider = network_provider(wl, theta)
    d = wl.dim
    n, nb = pts.shape[0], bpts.shape[0]
    cls, sides = S.classify(wl, pts, h)
    y = S.stencil_nodes(pts, h)
    r = np.zeros(n)
    req = {0: [], 1: []}           # side -> list of (row ids, X[m, d], dr/dU[m])
    # uncut cells -------------------------------------------------------------
    for s in (0, 1):
        ids = np.nonzero(cls == s)[0]
        if ids.size == 0:
            continue
        X = y[ids].reshape(-1, d)
        U = provider(s, X).reshape(ids.size, 2 * d + 1)
        r[ids] = S.uncut_residual(wl, prob, pts[ids], h, U, s)
        coef = S.uncut_residual_dU(wl, prob, pts[ids], h, s)
        req[s].append((np.repeat(ids, 2 * d + 1), X, coef.ravel()))
    # cut cells -----------------------------------------------------------------
    ids = np.nonzero(cls == S.CLASS_CUT)[0]
    if ids.size:
        yc = y[ids]                                   # [m, 2d+1, d]
        sc = sides[ids]
        U = np.empty(sc.shape)
        for s, mask in ((0, sc), (1, ~sc)):
            if mask.any():
                U[mask] = provider(s, yc[mask])
        glo = None
        lo = S.lo_side(wl)
        if lo >= 0 and glo_override is not None:
            glo = glo_override
        elif lo >= 0:
            glo = np.zeros(yc.shape)
            for a in range(d):
                e = np.zeros(d)
                e[a] = h
                up = provider(lo, (yc + e).reshape(-1, d)).reshape(sc.shape)
                dn = provider(lo, (yc - e).reshape(-1, d)).reshape(sc.shape)
                glo[..., a] = (up - dn) / (2 * h)
        J = S.jump_extension(wl, prob, yc, glo)
        terms = S.cut_terms(wl, prob, pts[ids], h, sc, J)
        r[ids] = S.cut_residual(U, terms, h)
        coef = S.cut_residual_dU(terms, h)
        res_glo = glo
        for s, mask in ((0, sc), (1, ~sc)):
            if mask.any():
                rows = np.repeat(ids[:, None], 2 * d + 1, axis=1)[mask]
                req[s].append((rows, yc[mask], coef[mask]))
    # boundary points ------------------------------------------------------------
    sb = G.side_minus(wl, bpts)
    Ub = np.empty(nb)
    for s, mask in ((0, sb), (1, ~sb)):
        if mask.any():
            Ub[mask] = provider(s, bpts[mask])
    rb = S.boundary_residual(wl, prob, bpts, h, Ub)
    loss = (np.dot(r, r) + np.dot(rb, rb)) / (n + nb)
    return {"r": r, "rb": rb, "cls": cls, "loss": loss, "req": req, "sb": sb, "nets": nets,
            "glo": res_glo if ids.size else None}


def level_spacings(wl: I.Workload):
    """Cell sides of the resolution levels: h, h/2, ..., h/2^levels (paper
    Sec. 3: implicit cells of several resolutions at each collocation point;
    Sec. 4.2: a base resolution implicitly refined)."""
    return [wl.h / 2.0 ** l for l in range(wl.levels + 1)]


def multires_loss(wl: I.Workload, theta: np.ndarray, pts: np.ndarray, bpts: np.ndarray):
    """Loss over every resolution level: the sum of the levels' losses."""
    return sum(residuals(wl, theta, pts, bpts, h=hl)["loss"] for hl in level_spacings(wl))


def loss_and_grad(wl: I.Workload, theta: np.ndarray, pts: np.ndarray, bpts: np.ndarray,
                  h: float = None, dL: float = 1.0, glo_override=None, abs_residual: bool = False):
    """Loss and dL/dtheta (FP64).  dL scales the gradient (upstream factor).
    Without an explicit h, a workload with refinement levels sums the loss
    and gradient over h, h/2, ..., h/2^levels; the returned dict then holds
    the base level's classes and "r_levels", every level's interior and
    boundary residuals, level-major.  abs_residual=True returns instead
    sum_p (2 |r_p| / (N + N_b)) d r_p / d theta, the gradient with the
    residuals' signs removed: a scale for how large the gradient's terms are
    where their signs cancel (test infrastructure: rounding bars)."""
    if h is None and wl.levels > 0:
        L, g, out = 0.0, None, None
        rl = []
        for hl in level_spacings(wl):
            Ll, gl, res = loss_and_grad(wl, theta, pts, bpts, h=hl, dL=dL, abs_residual=abs_residual)
            L += Ll
            g = gl if g is None else g + gl
            out = res if out is None else out
            rl.append(np.concatenate([res["r"], res["rb"]]))
        out = dict(out)
        out["r_levels"] = np.concatenate(rl)
        return L, g, out
    h = wl.h if h is None else h
    res = residuals(wl, theta, pts, bpts, h, glo_override=glo_override)
    d = wl.dim
    n, nb = pts.shape[0], bpts.shape[0]
    scale = 2.0 * dL / (n + nb)
    rbar = scale * (np.abs(res["r"]) if abs_residual else res["r"])
    rbbar = scale * (np.abs(res["rb"]) if abs_residual else res["rb"])
    grads = []
    for s in (0, 1):
        Xs, Ws = [], []
        for rows, X, coef in res["req"][s]:
            Xs.append(X)
            Ws.append(rbar[rows] * coef)
        mb = res["sb"] if s == 0 else ~res["sb"]
        if mb.any():
            Xs.append(bpts[mb])
            Ws.append(rbbar[mb] * (2 * d / (h * h)))
        X = np.concatenate(Xs) if Xs else np.zeros((0, d))
        Wt = np.concatenate(Ws) if Ws else np.zeros(0)
        grads.append(_grad_net(wl, res["nets"][s], X, Wt))
    return res["loss"], np.concatenate(grads), res


def adam_step(theta, m, v, g, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """Bias-corrected Adam (Kingma & Ba 2014), FP64, returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
