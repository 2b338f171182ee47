"""Pins of the oracle's NBM step: finite differences of the loss, parameter
counts (982 for the two 5x10 sine nets of the paper's Sec. 4.1), Adam's
closed-form first step, Philox known-answer vectors and sampler properties."""
import os

import numpy as np
import pytest

import nbm_inputs as I
from oracle import mlp as M
from oracle import nbm as N
from oracle import philox as P
from oracle import scheme as S


def test_param_counts():
    assert I.C1.n_params == 674
    assert I.C2.n_params == 17282
    assert I.C3.n_params == 100354 and I.C4.n_params == 100354
    paper = I.C2.replace(width=10, depth=5, act=I.ACT_SIN)
    assert paper.n_params == 982
    th = I.xavier_params(paper, 0)
    nets = M.unpack(paper, th)
    assert len(nets[0]) == 6 and nets[0][0][0].shape == (10, 3) and nets[0][1][0].shape == (10, 10)


def _fd_check(wl, th, pts, bpts, idx, glo=None, rtol=1e-6):
    L, g, res = N.loss_and_grad(wl, th, pts, bpts, glo_override=glo)
    for j in idx:
        e = np.zeros_like(th)
        step = 1e-6 * max(1.0, abs(th[j]))
        e[j] = step
        lp = N.residuals(wl, th + e, pts, bpts, glo_override=glo)["loss"]
        lm = N.residuals(wl, th - e, pts, bpts, glo_override=glo)["loss"]
        fd = (lp - lm) / (2 * step)
        assert abs(g[j] - fd) <= rtol * max(abs(fd), 1e-3 * np.abs(g).max()), (j, g[j], fd)
    return res


@pytest.mark.parametrize("wlname,act", [("c1", I.ACT_TANH), ("c1", I.ACT_SIN), ("c2", I.ACT_TANH),
                                        ("c3", I.ACT_SIN)])
def test_gradient_finite_differences(wlname, act):
    base = I.WORKLOADS[wlname]
    wl = base.replace(width=6, depth=3, act=act, h=1.0 / 16)
    th = I.xavier_params(wl, 0) * 1.5
    pts, bpts = I.collocation_batch(wl, 96, 12, seed=5)
    pts = np.concatenate([pts, I.near_interface_points(wl, 24, 0.05, seed=6)])
    rng = np.random.default_rng(0)
    idx = rng.choice(th.size, 12, replace=False)
    glo = None
    if S.lo_side(wl) >= 0:
        glo = N.residuals(wl, th, pts, bpts)["glo"]
    res = _fd_check(wl, th, pts, bpts, idx, glo=glo)
    assert (res["cls"] == S.CLASS_CUT).sum() > 5
    assert (res["cls"] == S.CLASS_A_MINUS).sum() > 0 and (res["cls"] == S.CLASS_A_PLUS).sum() > 0


def test_stop_gradient_on_lagged_term():
    """With a contrast the lagged low-mu derivative is held constant: the
    gradient differs from the full derivative only through the low-mu net."""
    wl = I.C2.replace(width=6, depth=2, h=1.0 / 16)
    th = I.xavier_params(wl, 0)
    pts = I.near_interface_points(wl, 40, 0.04, seed=2)
    bpts = np.zeros((0, 3))
    _, g, _ = N.loss_and_grad(wl, th, pts, bpts)
    pn = wl.params_per_net
    j = pn + 3   # a parameter of the high-mu (plus) network
    e = np.zeros_like(th)
    e[j] = 1e-6
    fd = (N.residuals(wl, th + e, pts, bpts)["loss"] - N.residuals(wl, th - e, pts, bpts)["loss"]) / 2e-6
    assert g[j] == pytest.approx(fd, rel=1e-6)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(1)
    th = rng.normal(size=50)
    g = rng.normal(size=50)
    new, m, v = N.adam_step(th, np.zeros(50), np.zeros(50), g, 1, lr=1e-3)
    assert np.allclose(new - th, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)


def test_philox_known_answers():
    # published known-answer vectors of the generator (fixture cites its source)
    path = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")
    tv = []
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            w = [int(x, 16) for x in line.split()]
            tv.append((w[0:4], w[4:6], w[6:10]))
    assert len(tv) == 3
    for c, k, e in tv:
        r = P.philox4x32_10(np.array(c, dtype=np.uint32), np.array(k, dtype=np.uint32))
        assert [int(x) for x in r] == list(e)


def test_sampler_lattice_and_ranges():
    pts, bpts = P.sample_points(3, 1.0 / 128, 20000, 600, seed=1234, step=7)
    q = 2.0 ** 22
    assert np.all(pts * q == np.round(pts * q)) and np.all(bpts * q == np.round(bpts * q))
    assert pts.min() >= -1 + 1 / 128 and pts.max() <= 1 - 1 / 128
    assert abs(pts.mean()) < 0.02 and abs(pts.std() - np.sqrt((2 - 2 / 128) ** 2 / 12)) < 0.01
    on_face = np.isclose(np.abs(bpts), 1.0).sum(axis=1)
    assert np.all(on_face >= 1)
    p2, _ = P.sample_points(3, 1.0 / 128, 20000, 600, seed=1234, step=8)
    assert not np.array_equal(pts, p2)
    p3, b3 = P.sample_points(3, 1.0 / 128, 20000, 600, seed=1234, step=7)
    assert np.array_equal(pts, p3) and np.array_equal(bpts, b3)


def test_loss_is_mean_square():
    wl = I.C1.replace(width=4)
    th = I.xavier_params(wl, 0)
    pts, bpts = I.collocation_batch(wl, 64, 8)
    res = N.residuals(wl, th, pts, bpts)
    assert res["loss"] == pytest.approx((np.sum(res["r"] ** 2) + np.sum(res["rb"] ** 2)) / 72, rel=1e-15)


def test_multiresolution_gradient_finite_differences():
    """Three refinement levels (cells of side h, h/2, h/4, h/8 at every point,
    losses summed): the gradient matches central differences of the summed
    loss, and each level sees its own cut cells."""
    wl = I.C1.replace(width=6, depth=2, act=I.ACT_SIN, h=1.0 / 8, levels=3)
    th = I.xavier_params(wl, 1) * 1.5
    pts, bpts = I.collocation_batch(wl, 80, 10, seed=7)
    pts = np.concatenate([pts, I.near_interface_points(wl, 40, 0.1, seed=8)])
    L, g, res = N.loss_and_grad(wl, th, pts, bpts)
    assert res["r_levels"].shape == (4 * (pts.shape[0] + bpts.shape[0]),)
    cuts = [(N.residuals(wl, th, pts, bpts, h=hl)["cls"] == S.CLASS_CUT).sum() for hl in N.level_spacings(wl)]
    assert cuts[0] > cuts[-1] > 0
    assert abs(L - N.multires_loss(wl, th, pts, bpts)) <= 1e-12 * L
    rng = np.random.default_rng(1)
    for j in rng.choice(th.size, 10, replace=False):
        e = np.zeros_like(th)
        step = 1e-6 * max(1.0, abs(th[j]))
        e[j] = step
        fd = (N.multires_loss(wl, th + e, pts, bpts) - N.multires_loss(wl, th - e, pts, bpts)) / (2 * step)
        assert abs(g[j] - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(g).max()), (j, g[j], fd)


@pytest.mark.parametrize("mu_plus", [1.0, 10.0])
def test_helmholtz_gradient_finite_differences(mu_plus):
    """With k^- = 2, k^+ = 5 the centre value enters every residual: the
    gradient still matches central differences (lagged term held fixed)."""
    wl = I.C2.replace(width=6, depth=2, act=I.ACT_SIN, h=1.0 / 16, mu_plus=mu_plus, k_minus=2.0, k_plus=5.0)
    th = I.xavier_params(wl, 3) * 1.5
    pts, bpts = I.collocation_batch(wl, 60, 8, seed=9)
    pts = np.concatenate([pts, I.near_interface_points(wl, 30, 0.05, seed=10)])
    glo = N.residuals(wl, th, pts, bpts)["glo"] if S.lo_side(wl) >= 0 else None
    rng = np.random.default_rng(2)
    res = _fd_check(wl, th, pts, bpts, rng.choice(th.size, 10, replace=False), glo=glo)
    assert (res["cls"] == S.CLASS_CUT).sum() > 5


def test_helmholtz_uncut_residual_of_the_exact_solution_is_second_order():
    wl = I.C2.replace(k_minus=2.0, k_plus=5.0)
    pts, _ = I.collocation_batch(wl, 3000, 0, seed=4)
    rms = []
    for h in (1 / 16, 1 / 32, 1 / 64):
        res = N.residuals(wl, None, pts, np.zeros((0, 3)), h=h, provider=N.exact_provider(wl))
        m = res["cls"] != S.CLASS_CUT
        rms.append(np.sqrt(np.mean(res["r"][m] ** 2)))
    assert rms[0] / rms[1] > 3.5 and rms[1] / rms[2] > 3.5


def test_variable_mu_gradient_finite_differences():
    """The Sec. 4.1 coefficients (face-centre mu in every row, mu at the
    projection point in the jump extension): gradient against central
    differences on tiny sine nets (lagged term held fixed)."""
    wl = I.PAPER.replace(width=5, depth=3, h=1.0 / 16)
    th = I.xavier_params(wl, 4) * 1.5
    pts, bpts = I.collocation_batch(wl, 60, 8, seed=11)
    pts = np.concatenate([pts, I.near_interface_points(wl, 30, 0.05, seed=12)])
    glo = N.residuals(wl, th, pts, bpts)["glo"]
    rng = np.random.default_rng(3)
    res = _fd_check(wl, th, pts, bpts, rng.choice(th.size, 10, replace=False), glo=glo)
    assert (res["cls"] == S.CLASS_CUT).sum() > 5


def test_variable_mu_exact_solution_residual_second_order():
    wl = I.PAPER
    pts, _ = I.collocation_batch(wl, 3000, 0, seed=4)
    rms = []
    for h in (1 / 16, 1 / 32, 1 / 64):
        res = N.residuals(wl, None, pts, np.zeros((0, 3)), h=h, provider=N.exact_provider(wl))
        m = res["cls"] != S.CLASS_CUT
        rms.append(np.sqrt(np.mean(res["r"][m] ** 2)))
    assert rms[0] / rms[1] > 3.5 and rms[1] / rms[2] > 3.5, rms
