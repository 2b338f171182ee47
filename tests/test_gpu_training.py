"""End-to-end training on the GPU through the C ABI: the loss falls, the
trained surrogate approaches the closed-form solution, the BF16-operand form
stays within the FP32 form's error, and the learned surrogate beats the
method without it (the grid solution interpolated off the grid) at points next
to the interface."""
import numpy as np
import pytest

import nbm_inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _train(wl, steps):
    from paper_2210_14907_amd.train import train
    params, nbm, state, losses = train(wl, steps=steps, seed=1)
    return params, nbm, losses.numpy()


def _judge_errors(wl, params, nbm, n=64):
    from oracle import grid as OG
    gs = OG.GridSystem(wl, n)
    U = gs.solve()
    x = gs.x[gs.interior]
    u = nbm.eval(params, torch.tensor(x, dtype=torch.float32, device=nbm.device)).cpu().numpy()
    ex = gs.prob.u_exact(x)
    return np.abs(u - ex).max(), np.sqrt(np.mean((u - ex) ** 2)), gs, U


_CACHE = {}


def _trained(name, wl, steps):
    if name not in _CACHE:
        _CACHE[name] = _train(wl, steps)
    return _CACHE[name]


def test_c1_training_reduces_loss():
    params, nbm, losses = _trained("c1", I.C1, I.C1.steps)
    print(f"[train] c1 loss {losses[0]:.3e} -> {losses[-1]:.3e}", flush=True)
    assert np.all(np.isfinite(losses))
    assert losses[-20:].mean() < 0.5 * losses[:20].mean()


def test_c2_fp32_accuracy_and_bf16_ratio():
    p32, n32, l32 = _trained("c2", I.C2, I.C2.steps)
    p16, n16, l16 = _trained("c2_bf16", I.C2.replace(prec=I.PREC_BF16), I.C2.steps)
    e32, r32, _, _ = _judge_errors(I.C2, p32, n32)
    e16, r16, _, _ = _judge_errors(I.C2, p16, n16)
    print(f"[train] c2 fp32 Linf {e32:.3e} L2 {r32:.3e} | bf16 Linf {e16:.3e} L2 {r16:.3e} "
          f"ratio {e16 / e32:.2f}", flush=True)
    assert l32[-20:].mean() < 0.05 * l32[:20].mean()
    assert e32 < 0.5
    assert e16 <= 1.5 * e32


def test_learned_surrogate_beats_interpolated_grid_near_interface():
    """At random off-grid points within two judge cells of the interface the
    two-network surrogate keeps the jump sharp; multilinear interpolation of
    the grid solution (the method without the learned part) smears it."""
    from oracle import geometry as G
    from oracle import grid as OG
    wl = I.C2
    params, nbm, _ = _trained("c2", wl, wl.steps)
    _, _, gs, U = _judge_errors(wl, params, nbm)
    rng = np.random.default_rng(7)
    v = rng.normal(size=(100000, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    x = v * (wl.radius + rng.uniform(-2 * gs.h, 2 * gs.h, size=(100000, 1)))
    ex = gs.prob.u_exact(x)
    u = nbm.eval(params, torch.tensor(x, dtype=torch.float32, device=nbm.device)).cpu().numpy()
    ui = OG.interp_grid(U, gs.n, 3, x)
    e_net, e_int = np.abs(u - ex).max(), np.abs(ui - ex).max()
    print(f"[gain] near-interface Linf: surrogate {e_net:.3e} vs interpolated grid {e_int:.3e}; "
          f"memory {4 * nbm.P / 1e3:.0f} KB vs {8 * U.size / 1e6:.1f} MB", flush=True)
    assert e_net < e_int
