"""Cut-cell finite-volume residual at arbitrary cell centres (oracle, FP64).

Paper Sec. 3: an implicit compute cell of a given resolution is placed at each
collocation point, the solution values at the stencil vertices come from the
networks, and each point contributes r_p = |M^-1 A u - M^-1 b|.  The paper's
loss equation and the coefficients of the bootstrapped scheme are not in the
text, so the scheme below is this project's reading of them:

  cell C_p = x_p + [-h/2, h/2]^d, nodes y_0 = x_p, y_(+-i) = x_p +- h e_i;
  U(y) = u^{sigma(y)}(y);  two-sided values u~^s(y) = U(y) (+-) J(y) when y is
  on the other side, J(y) = alpha(pi(y)) + dist(y) * j (jump extension);
  R_p = -(1/h^2) sum_F sum_s mu^s a^s_F [u~^s(y_F) - u~^s(y_0)]
        + sum_s k^s v^s u~^s(y_0) - sum_s v^s f^s(x_p) + gamma_p beta(pi(c_p)) / h;
  r_p = R_p / mubar_p, mubar_p = (1/2d) sum_F sum_s mu^s a^s_F   (Jacobi M^-1).

Uncut cells (every node and corner on one side s) reduce to
r_p = -sum_i (U(y_+i) - 2 U(y_0) + U(y_-i)) / h^2 + (k^s U(y_0) - f^s(x_p)) / mu^s.
Node order everywhere: 0 = centre, 1 + 2i = +e_i, 2 + 2i = -e_i; face F = 2i
(+e_i) and 2i + 1 (-e_i) pairs with node 1 + F.
"""
from __future__ import annotations

import numpy as np

import nbm_inputs as I
from . import geometry as G
from .problems import Problem

CLASS_A_MINUS = 0
CLASS_A_PLUS = 1
CLASS_CUT = 2


def stencil_nodes(xc: np.ndarray, h: float) -> np.ndarray:
    """Nodes y[n, 2d+1, d] of the cells centred at xc[n, d]."""
    n, d = xc.shape
    y = np.repeat(xc[:, None, :], 2 * d + 1, axis=1)
    for i in range(d):
        y[:, 1 + 2 * i, i] += h
        y[:, 2 + 2 * i, i] -= h
    return y


def classify(wl: I.Workload, xc: np.ndarray, h: float):
    """Class of each cell: all nodes and corners in Omega^- (0), all in
    Omega^+ (1), mixed (2).  Also returns node sides (True = minus)."""
    d = wl.dim
    y = stencil_nodes(xc, h)
    corners = xc[:, None, :] + h * G.corner_offsets(d)[None, :, :]
    sn = G.side_minus(wl, y)
    sc = G.side_minus(wl, corners)
    allm = sn.all(axis=1) & sc.all(axis=1)
    allp = (~sn).all(axis=1) & (~sc).all(axis=1)
    cls = np.full(xc.shape[0], CLASS_CUT, dtype=np.int64)
    cls[allm] = CLASS_A_MINUS
    cls[allp] = CLASS_A_PLUS
    return cls, sn


def lo_side(wl: I.Workload) -> int:
    """Side with the smaller diffusion coefficient (0 = minus), or -1 if equal.
    With the variable coefficients of Sec. 4.1, mu^+ = e^-z <= e < 4 <= mu^-
    on the whole box, and the constants mu_minus > mu_plus record that."""
    if wl.mu_minus == wl.mu_plus:
        return -1
    return 0 if wl.mu_minus < wl.mu_plus else 1


def face_centres(xc: np.ndarray, h: float) -> np.ndarray:
    """Centres x_p +- (h/2) e_a of the 2d faces, order +e_0, -e_0, +e_1, ..."""
    n, d = xc.shape
    xf = np.repeat(xc[:, None, :], 2 * d, axis=1)
    for a in range(d):
        xf[:, 2 * a, a] += 0.5 * h
        xf[:, 2 * a + 1, a] -= 0.5 * h
    return xf


def jump_data(wl: I.Workload, prob: Problem, y: np.ndarray):
    """Interface data the jump extension needs at nodes y[..., d]: the
    projection pi(y) (one Newton step), the signed distance, the normal at
    pi(y), alpha and beta there."""
    pi, dist, n = G.project(wl, y)
    return {"alpha": prob.alpha(pi, n), "beta": prob.beta(pi, n), "dist": dist, "n": n,
            "mu_m": prob.mu_at(0, pi), "mu_p": prob.mu_at(1, pi)}


def jump_extension(wl: I.Workload, prob: Problem, y: np.ndarray, grad_lo: np.ndarray = None,
                   data=None):
    """J(y) = alpha(pi(y)) + dist(y) * j, an extension of [u] = u^+ - u^- off Gamma.

    j approximates [d_n u] from mu^+ d_n u^+ - mu^- d_n u^- = beta:
      equal mu:  j = beta / mu;
      lo = minus: j = beta/mu^+ + (mu^-/mu^+ - 1) g,
      lo = plus:  j = beta/mu^- + (1 - mu^+/mu^-) g,
    with g = n(pi(y)) . grad_lo(y), the lagged normal derivative on the side
    with the smaller coefficient (|1 - mu_lo/mu_hi| < 1), and mu^-+ taken at
    pi(y).  grad_lo[..., d] is supplied by the caller (central differences of
    the lo-side field).  data = jump_data(wl, prob, y) may be passed instead
    of y."""
    if data is None:
        data = jump_data(wl, prob, y)
    al, be, dist, n = data["alpha"], data["beta"], data["dist"], data["n"]
    mm, mp = data["mu_m"], data["mu_p"]
    lo = lo_side(wl)
    if lo < 0:
        j = be / mm
    else:
        gl = (grad_lo * n).sum(axis=-1)
        j = be / mp + (mm / mp - 1.0) * gl if lo == 0 else be / mm + (1.0 - mp / mm) * gl
    return al + dist * j


def cut_static(wl: I.Workload, prob: Problem, xc: np.ndarray, h: float, fvals=None):
    """The parts of the cut-cell residual that depend on neither U nor J:
    geometry, face coefficients c[n, 2d] (sum_s mu^s a^s_F), mubar[n], the
    source sum_s v^s f^s(x_p) and the interface term gamma_p beta(pi(c_p))/h.
    fvals = (f^-(xc), f^+(xc)) may be passed in precomputed."""
    d = wl.dim
    geom = G.cell_geometry(wl, xc, h)
    xf = face_centres(xc, h)
    an = geom["aneg"]
    ap = 1.0 - an
    # mu^s a^s_F with mu^s at the face centre
    cm, cp = prob.mu_at(0, xf) * an, prob.mu_at(1, xf) * ap
    c = cm + cp
    mubar = c.sum(axis=1) / (2 * d)
    vneg = geom["vneg"]
    fm, fp = (prob.f_side(0, xc), prob.f_side(1, xc)) if fvals is None else fvals
    src = vneg * fm + (1.0 - vneg) * fp
    pic, _, nc = G.project(wl, geom["cen"])
    bterm = np.where(geom["gamma"] > 0, geom["gamma"] * prob.beta(pic, nc) / h, 0.0)
    # Helmholtz weights k^s v^s of the two-sided centre values
    km, kp = wl.k_minus * vneg, wl.k_plus * (1.0 - vneg)
    return {"c": c, "mubar": mubar, "cm": cm, "cp": cp, "src": src, "bterm": bterm, "geom": geom,
            "km": km, "kp": kp}


def cut_terms(wl: I.Workload, prob: Problem, xc: np.ndarray, h: float, sides: np.ndarray,
              J: np.ndarray, static=None):
    """Everything of the cut-cell residual that does not depend on U.

    sides[n, 2d+1] node sides (True = minus), J[n, 2d+1] jump extension at the
    nodes.  Returns dict with face coefficients c[n, 2d] (sum_s mu^s a^s_F),
    mubar[n], the constant part K[n] of R_p (so that
    R_p = -(1/h^2) sum_F c_F (U_F - U_0) + K) and the geometry.  static =
    cut_static(...) of the same cells may be passed in."""
    d = wl.dim
    st = cut_static(wl, prob, xc, h) if static is None else static
    cm, cp = st["cm"], st["cp"]
    # corrections u~^s(y) - U(y)
    corr_m = np.where(sides, 0.0, -J)
    corr_p = np.where(sides, J, 0.0)
    flux_corr = np.zeros(xc.shape[0])
    for F in range(2 * d):
        flux_corr += cm[:, F] * (corr_m[:, 1 + F] - corr_m[:, 0])
        flux_corr += cp[:, F] * (corr_p[:, 1 + F] - corr_p[:, 0])
    # sum_s k^s v^s u~^s(y_0) = (k^- v^- + k^+ v^+) U(y_0) + the corrections' part
    kcorr = st["km"] * corr_m[:, 0] + st["kp"] * corr_p[:, 0]
    K = -flux_corr / (h * h) + kcorr - st["src"] + st["bterm"]
    return {"c": st["c"], "mubar": st["mubar"], "K": K, "geom": st["geom"], "kap": st["km"] + st["kp"]}


def cut_residual(U: np.ndarray, terms, h: float) -> np.ndarray:
    """r_p = R_p / mubar_p with R_p = -(1/h^2) sum_F c_F (U_F - U_0) + kap U_0 + K."""
    c = terms["c"]
    R = terms["K"] + terms["kap"] * U[:, 0]
    for F in range(c.shape[1]):
        R -= c[:, F] * (U[:, 1 + F] - U[:, 0]) / (h * h)
    return R / terms["mubar"]


def cut_residual_dU(terms, h: float) -> np.ndarray:
    """d r_p / d U at the 2d+1 nodes (the residual is affine in U)."""
    c = terms["c"] / terms["mubar"][:, None] / (h * h)
    n, nf = c.shape
    out = np.zeros((n, nf + 1))
    out[:, 0] = c.sum(axis=1) + terms["kap"] / terms["mubar"]
    out[:, 1:] = -c
    return out


def uncut_residual(wl: I.Workload, prob: Problem, xc: np.ndarray, h: float, U: np.ndarray,
                   side: int) -> np.ndarray:
    """r_p = -sum_i (U(y_+i) - 2 U(y_0) + U(y_-i)) / h^2 + (k^s U(y_0) - f^s(x_p)) / mu^s
    for constant mu; with variable mu, r_p = R_p / mubar_p with
    R_p = -(1/h^2) sum_F mu^s(x_F) (U(y_F) - U(y_0)) + k^s U(y_0) - f^s(x_p)."""
    k = (wl.k_minus, wl.k_plus)[side]
    if wl.mu_kind != I.MU_CONST:
        muF = prob.mu_at(side, face_centres(xc, h))
        R = k * U[:, 0] - prob.f_side(side, xc)
        for F in range(2 * wl.dim):
            R = R - muF[:, F] * (U[:, 1 + F] - U[:, 0]) / (h * h)
        return R / (muF.sum(axis=1) / (2 * wl.dim))
    lap = np.zeros(xc.shape[0])
    for i in range(wl.dim):
        lap += U[:, 1 + 2 * i] - 2.0 * U[:, 0] + U[:, 2 + 2 * i]
    mu = (wl.mu_minus, wl.mu_plus)[side]
    r = -lap / (h * h) - prob.f_side(side, xc) / mu
    return r + (k / mu) * U[:, 0] if k else r


def uncut_residual_dU(wl: I.Workload, prob: Problem, xc: np.ndarray, h: float, side: int) -> np.ndarray:
    """d r_p / d U at the 2d+1 nodes of uncut cells (the residual is affine in U)."""
    d = wl.dim
    k = (wl.k_minus, wl.k_plus)[side]
    if wl.mu_kind != I.MU_CONST:
        muF = prob.mu_at(side, face_centres(xc, h))
        mubar = muF.sum(axis=1) / (2 * d)
        out = np.empty((xc.shape[0], 2 * d + 1))
        out[:, 1:] = -muF / (h * h) / mubar[:, None]
        out[:, 0] = (muF.sum(axis=1) / (h * h) + k) / mubar
        return out
    mu = (wl.mu_minus, wl.mu_plus)[side]
    out = np.full((xc.shape[0], 2 * d + 1), -1.0 / (h * h))
    out[:, 0] = 2.0 * d / (h * h) + k / mu
    return out


def boundary_residual(wl: I.Workload, prob: Problem, xb: np.ndarray, h: float,
                      Ub: np.ndarray) -> np.ndarray:
    """Dirichlet rows at boundary points: r_b = (2d/h^2)(U(x_b) - g(x_b))."""
    return (2 * wl.dim / (h * h)) * (Ub - prob.g(xb))
