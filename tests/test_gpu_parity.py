"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.  Bars: FP32 operands rel <= 1e-5, BF16 operands
rel <= 2e-2 (loss, residual vector, gradient)."""
import math

import numpy as np
import pytest

import nbm_inputs as I
from oracle import nbm as N
from oracle import philox as PH
from oracle import scheme as S
from tests.gpu_common import max_rel, parity_batch, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {I.PREC_FP32: 1e-5, I.PREC_BF16: 2e-2}


def _nbm(wl, n, nb, **kw):
    from paper_2210_14907_amd import NBM
    return NBM(wl, max_points=max(n, 16), max_boundary=max(nb, 1), **kw)


def _run(wl, pts, bpts, theta, **kw):
    dev = torch.device("cuda:0")
    m = _nbm(wl, pts.shape[0], bpts.shape[0], **kw)
    p = torch.tensor(theta, dtype=torch.float32, device=dev)
    tp = torch.tensor(pts, dtype=torch.float32, device=dev)
    tb = torch.tensor(bpts, dtype=torch.float32, device=dev).reshape(-1, wl.dim)
    loss, res, grad = m.forward_residual(p, tp, tb, want_residual=True, want_grad=True)
    counts = m.batch_counts().cpu().numpy()
    torch.cuda.synchronize()
    return loss.item(), res.cpu().numpy(), grad.cpu().numpy(), counts, m


CASES = [
    # name, workload, n, nb, n_near, band
    ("c1", I.C1, 4096, 256, 256, 0.05),
    ("c2", I.C2, 4096, 96, 512, 0.02),
    ("c3", I.C3, 2048, 48, 256, 0.01),
    ("c4", I.C4, 2048, 48, 256, 0.004),
    ("c3_fp32", I.C3.replace(prec=I.PREC_FP32), 2048, 48, 256, 0.01),
    ("c2_bf16", I.C2.replace(prec=I.PREC_BF16), 4096, 96, 512, 0.02),
    # equal coefficients: no low-mu neighbour centres on the fused path
    ("c2_equal_mu", I.C2.replace(mu_plus=1.0), 4096, 96, 512, 0.02),
    # Helmholtz term k u (paper Sec. 2): fused W = 64, two-pass W = 128 in both
    # operand precisions, layered W = 16
    ("c2_helmholtz", I.C2.replace(k_minus=2.0, k_plus=5.0), 4096, 96, 512, 0.02),
    ("c3_helmholtz_fp32", I.C3.replace(prec=I.PREC_FP32, k_minus=2.0, k_plus=5.0), 2048, 48, 256, 0.01),
    ("c3_helmholtz_bf16", I.C3.replace(k_minus=2.0, k_plus=5.0), 2048, 48, 256, 0.01),
    ("c1_helmholtz", I.C1.replace(k_minus=3.0, k_plus=1.0), 4096, 256, 256, 0.05),
    ("c4_helmholtz", I.C4.replace(k_minus=4.0, k_plus=0.5), 2048, 48, 256, 0.004),
    # level set stored on a coarse mesh (the star sampled on 32^3 nodes), with
    # the Helmholtz term: the manufactured sphere-problem data on that interface
    ("c2_mesh_star_helmholtz", I.C2.replace(interface=I.IFACE_GRID, phi_shape=I.IFACE_STAR, phi_n=32,
                                            star_amp=0.1, k_minus=2.0, k_plus=5.0), 4096, 96, 512, 0.01),
    ("c4_mesh_star", I.C4.replace(interface=I.IFACE_GRID, phi_shape=I.IFACE_STAR, phi_n=32), 2048, 48, 256, 0.004),
]


@pytest.mark.parametrize("name,wl,n,nb,n_near,band", CASES, ids=[c[0] for c in CASES])
def test_step_parity(name, wl, n, nb, n_near, band):
    print(f"[parity] {name} n={n}+{n_near} nb={nb}", flush=True)
    theta = I.xavier_params(wl, 0)
    pts, bpts = parity_batch(wl, n, nb, n_near, band)
    # points are FP32 on the GPU: give the oracle the identical values
    pts = pts.astype(np.float32).astype(np.float64)
    bpts = bpts.astype(np.float32).astype(np.float64)
    th32 = theta.astype(np.float32).astype(np.float64)
    L_o, g_o, res_o = N.loss_and_grad(wl, th32, pts, bpts)
    L_g, r_g, g_g, counts, _ = _run(wl, pts, bpts, th32)
    cls = res_o["cls"]
    ncut = int((cls == S.CLASS_CUT).sum())
    assert counts[0] == (cls == 0).sum() and counts[1] == (cls == 1).sum() and counts[2] == ncut
    assert ncut > 0 and counts[5] == 0
    # the 128-wide pass takes its fast form at these arguments (no fallback)
    assert counts[6] == 0
    tol = TOL[wl.prec]
    r_o = np.concatenate([res_o["r"], res_o["rb"]])
    e_loss = abs(L_g - L_o) / abs(L_o)
    e_res = max_rel(r_g, r_o)
    e_grad = rel_err(g_g, g_o)
    # uncut residuals on their own scale
    un = np.nonzero(cls != S.CLASS_CUT)[0]
    e_unc = max_rel(r_g[un], res_o["r"][un])
    print(f"[parity] {name}: loss {e_loss:.2e} res {e_res:.2e} uncut {e_unc:.2e} grad {e_grad:.2e} "
          f"(cut {ncut})", flush=True)
    assert e_loss <= tol and e_res <= tol and e_grad <= tol
    assert e_unc <= (5 * tol if wl.prec == I.PREC_FP32 else tol)


def test_step_parity_many_cut_cells():
    """More cut cells than the residual launch's 1,024 cut-cell blocks and
    more non-inline tiles than the forward-only pass's 512 blocks: both walk
    their work with the grid as stride, checked against the oracle."""
    wl = I.C2
    theta = I.xavier_params(wl, 2).astype(np.float32).astype(np.float64)
    pts, bpts = parity_batch(wl, 2048, 64, 2600, 0.003, seed=21)
    pts = pts.astype(np.float32).astype(np.float64)
    bpts = bpts.astype(np.float32).astype(np.float64)
    L_o, g_o, res_o = N.loss_and_grad(wl, theta, pts, bpts)
    L_g, r_g, g_g, counts, _ = _run(wl, pts, bpts, theta, cut_capacity=pts.shape[0])
    ncut = int((res_o["cls"] == S.CLASS_CUT).sum())
    nonin_tiles = ((2 + 2 * wl.dim) * ncut + bpts.shape[0]) // 16
    assert counts[2] == ncut and counts[5] == 0
    assert ncut > 1024 and nonin_tiles > 512
    r_o = np.concatenate([res_o["r"], res_o["rb"]])
    e_loss, e_res, e_grad = abs(L_g - L_o) / abs(L_o), max_rel(r_g, r_o), rel_err(g_g, g_o)
    print(f"[parity] c2_many_cut: loss {e_loss:.2e} res {e_res:.2e} grad {e_grad:.2e} (cut {ncut})", flush=True)
    tol = TOL[wl.prec]
    assert e_loss <= tol and e_res <= tol and e_grad <= tol


LARGE_ARG_CASES = [
    # name, workload, weight gain, n, nb, n_near, band
    ("c2_x8", I.C2, 8.0, 2048, 64, 256, 0.02),
    ("c3_fp32_x4", I.C3.replace(prec=I.PREC_FP32), 4.0, 2048, 64, 256, 0.01),
    ("c3_bf16_x4", I.C3, 4.0, 2048, 64, 256, 0.01),
    ("c1_x4", I.C1, 4.0, 4096, 256, 256, 0.05),
]


@pytest.mark.parametrize("name,wl,gain,n,nb,n_near,band", LARGE_ARG_CASES,
                         ids=[c[0] for c in LARGE_ARG_CASES])
def test_step_parity_large_arguments(name, wl, gain, n, nb, n_near, band):
    """Weights scaled up so that the difference arguments leave the tiny
    series tier: the longer series and the library-function paths of the
    activation streams are checked against the oracle as well (the sin net
    at a smaller gain: the hardware sine of the base argument is accurate to
    ~1e-7 |z| absolute, sized for pre-activations of order 1-10)."""
    theta = (I.xavier_params(wl, 1) * gain).astype(np.float32).astype(np.float64)
    pts, bpts = parity_batch(wl, n, nb, n_near, band, seed=11)
    pts = pts.astype(np.float32).astype(np.float64)
    bpts = bpts.astype(np.float32).astype(np.float64)
    L_o, g_o, res_o = N.loss_and_grad(wl, theta, pts, bpts)
    L_g, r_g, g_g, counts, _ = _run(wl, pts, bpts, theta)
    r_o = np.concatenate([res_o["r"], res_o["rb"]])
    e_loss, e_res, e_grad = abs(L_g - L_o) / abs(L_o), max_rel(r_g, r_o), rel_err(g_g, g_o)
    print(f"[parity] {name}: loss {e_loss:.2e} res {e_res:.2e} grad {e_grad:.2e} fallback {counts[6]}",
          flush=True)
    # the 128-wide pass with BF16 operands leaves its fast form here and
    # recomputes with per-element tiers (FP32 runs the general form alone)
    assert counts[6] == (1 if wl.width == 128 and wl.prec == I.PREC_BF16 else 0)
    # larger arguments: the condition of the streams grows with the gain (the
    # C3 FP32 gradient error goes from 1.9e-7 at gain 1 to 5.7e-6 at gain 4,
    # 30x, and BF16 from 2.9e-3 to 5.7e-2), so the bar is ten times the
    # operand precision's step bar
    tol = 10 * TOL[wl.prec]
    assert e_loss <= tol and e_res <= tol and e_grad <= tol


@pytest.mark.parametrize("wl", [I.C2, I.C3.replace(prec=I.PREC_FP32), I.C2.replace(k_minus=2.0, k_plus=5.0)],
                         ids=["c2_fused", "c3_two_pass", "c2_fused_helmholtz"])
def test_fused_and_layered_paths_agree(monkeypatch, wl):
    """The fused kernels (W=64 one-pass, W=128 two-pass) and the layered
    forward/backward give the same step (all are also checked against the
    oracle above)."""
    theta = I.xavier_params(wl, 5).astype(np.float32)
    pts, bpts = parity_batch(wl, 2048, 96, 256, 0.02, seed=8)
    a = _run(wl, pts, bpts, theta)
    monkeypatch.setenv("NBM_NO_FUSED", "1")
    b = _run(wl, pts, bpts, theta)
    assert abs(a[0] - b[0]) <= 1e-6 * abs(b[0])
    assert max_rel(a[1], b[1]) <= 1e-6
    # 2e-6, not 1e-6: each path accumulates a work-group's dW over its tiles
    # in FP32 before the fixed-order FP64 reduction, but the fused kernels
    # (512 or 256 work-groups, all layers in one pass) and the layered path
    # (one launch per layer) deal the tiles to work-groups differently, so the
    # same FP32 terms are summed in different orders and groupings
    assert rel_err(a[2], b[2]) <= 2e-6


def test_determinism_bitwise():
    wl = I.C2
    theta = I.xavier_params(wl, 3).astype(np.float32)
    pts, bpts = parity_batch(wl, 4096, 96, 256, 0.02, seed=4)
    a = _run(wl, pts, bpts, theta)
    b = _run(wl, pts, bpts, theta)
    assert a[0] == b[0]
    assert np.array_equal(a[2], b[2]) and np.array_equal(a[1], b[1])


def test_sampling_matches_oracle_philox():
    from paper_2210_14907_amd import NBM
    for wl in (I.C1, I.C2, I.C4):
        m = NBM(wl, max_points=20000, max_boundary=700)
        seed, step = 0x123456789A, 77
        pts, bpts = m.sample_points(seed, step, 20000, 700)
        po, bo = PH.sample_points(wl.dim, wl.h, 20000, 700, seed, step)
        assert np.array_equal(pts.cpu().numpy().astype(np.float64), po)
        assert np.array_equal(bpts.cpu().numpy().astype(np.float64), bo)


def test_adam_matches_oracle():
    from paper_2210_14907_amd import NBM
    wl = I.C1
    m = NBM(wl, max_points=64, max_boundary=8)
    rng = np.random.default_rng(0)
    P = wl.n_params
    th = rng.normal(size=P).astype(np.float32)
    g = rng.normal(size=P).astype(np.float32)
    m0 = (0.1 * rng.normal(size=P)).astype(np.float32)
    v0 = np.abs(0.1 * rng.normal(size=P)).astype(np.float32)
    dev = torch.device("cuda:0")
    tp, tm, tv, tg = (torch.tensor(a, device=dev) for a in (th, m0, v0, g))
    m.adam_step(tp, tm, tv, tg, 5, lr=1e-3)
    ref, mr, vr = N.adam_step(th.astype(np.float64), m0.astype(np.float64), v0.astype(np.float64),
                              g.astype(np.float64), 5, lr=1e-3)
    assert np.allclose(tp.cpu().numpy(), ref, rtol=0, atol=1e-6)
    assert np.allclose(tm.cpu().numpy(), mr, rtol=1e-6, atol=1e-7)
    assert np.allclose(tv.cpu().numpy(), vr, rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("wl", [I.C1, I.C2, I.C3, I.C4], ids=["c1", "c2", "c3", "c4"])
def test_eval_matches_oracle(wl):
    from paper_2210_14907_amd import NBM
    from oracle import geometry as G
    from oracle import mlp as M
    theta = I.xavier_params(wl, 1).astype(np.float32).astype(np.float64)
    m = NBM(wl, max_points=5000, max_boundary=1)
    dev = torch.device("cuda:0")
    p = torch.tensor(theta, dtype=torch.float32, device=dev)
    q = I.lattice_points(3000, wl.dim, -1.0, 1.0, seed=5)
    u = m.eval(p, torch.tensor(q, dtype=torch.float32, device=dev)).cpu().numpy()
    ref = M.eval_two(wl, theta, q, G.side_minus(wl, q))
    tol = 1e-5 if wl.prec == I.PREC_FP32 else 2e-2
    assert max_rel(u, ref) <= tol
    # grid tile: points -1 + 2 i / grid_n
    gn = 16
    mt = gn ** wl.dim // 4
    ut = m.eval(p, None, m=mt, tile_index=2, grid_n=gn).cpu().numpy()
    idx = np.arange(2 * mt, 3 * mt)
    coords = np.stack([(idx // gn ** a) % gn for a in range(wl.dim)], axis=1)
    xq = -1.0 + 2.0 * coords / gn
    ref_t = M.eval_two(wl, theta, xq, G.side_minus(wl, xq))
    # grid points on Gamma (|phi| at rounding level) may take either network:
    # compare the unique ones, accept either side for the rest
    tie = np.abs(G.phi(wl, xq)) < 1e-12
    alt = M.eval_two(wl, theta, xq, ~G.side_minus(wl, xq))
    ok_tie = np.minimum(np.abs(ut - ref_t), np.abs(ut - alt)) <= tol * np.abs(ref_t).max()
    assert max_rel(ut[~tie], ref_t[~tie]) <= tol and ok_tie[tie].all()


def test_eval_two_level_scan_every_output():
    """More than 2048 blocks of 256 query points take the two-level offsets scan
    (chunks of 1024 block counts, a ragged last chunk and a ragged last block);
    every output is compared with the oracle, so each query is written once and
    by the net of its side."""
    from paper_2210_14907_amd import NBM
    from oracle import geometry as G
    from oracle import mlp as M
    wl = I.C2
    theta = I.xavier_params(wl, 4).astype(np.float32).astype(np.float64)
    mq = 2050 * 256 + 77
    print(f"[parity] eval two-level scan m={mq}", flush=True)
    m = NBM(wl, max_points=mq, max_boundary=1, eval_only=True)
    dev = torch.device("cuda:0")
    p = torch.tensor(theta, dtype=torch.float32, device=dev)
    q = I.lattice_points(mq, wl.dim, -1.0, 1.0, seed=9)
    u = m.eval(p, torch.tensor(q, dtype=torch.float32, device=dev)).cpu().numpy()
    side = G.side_minus(wl, q)
    ref = M.eval_two(wl, theta, q, side)
    assert 0 < side.sum() < mq
    # points within FP32 rounding of Gamma may take either network
    tie = np.abs(G.phi(wl, q)) < 1e-6
    alt = M.eval_two(wl, theta, q[tie], ~side[tie])
    assert max_rel(u[~tie], ref[~tie]) <= 1e-5
    scale = np.abs(ref).max()
    assert np.all(np.minimum(np.abs(u[tie] - ref[tie]), np.abs(u[tie] - alt)) <= 1e-5 * scale)


def test_eval_star_side_near_interface():
    """Queries within 3e-3 of the star interface, where the evaluation decides
    each side from FP32 level-set values outside a 1e-3 margin and from FP64
    inside it: every output is compared with the oracle (FP32 operands, so a
    query given the other network's value fails)."""
    from paper_2210_14907_amd import NBM
    from oracle import geometry as G
    from oracle import mlp as M
    wl = I.C4.replace(prec=I.PREC_FP32)
    theta = I.xavier_params(wl, 5).astype(np.float32).astype(np.float64)
    cand = I.lattice_points(4_000_000, 3, -1.0, 1.0, seed=11) * 0.7
    cand = np.round(cand * 2.0 ** 22) / 2.0 ** 22
    ph = G.phi(wl, cand)
    q = cand[np.abs(ph) < 3e-3][:40_000]
    ph = G.phi(wl, q)
    print(f"[parity] star side: {q.shape[0]} queries, {int((np.abs(ph) <= 1e-3).sum())} inside the margin",
          flush=True)
    assert q.shape[0] > 20_000 and (np.abs(ph) <= 1e-3).sum() > 5_000
    m = NBM(wl, max_points=q.shape[0], max_boundary=1, eval_only=True)
    dev = torch.device("cuda:0")
    p = torch.tensor(theta, dtype=torch.float32, device=dev)
    u = m.eval(p, torch.tensor(q, dtype=torch.float32, device=dev)).cpu().numpy()
    side = G.side_minus(wl, q)
    ref = M.eval_two(wl, theta, q, side)
    tie = np.abs(ph) < 1e-12
    assert max_rel(u[~tie], ref[~tie]) <= 1e-5


def test_edge_cases_small_and_ragged():
    wl = I.C2
    theta = I.xavier_params(wl, 2).astype(np.float32).astype(np.float64)
    for n, nb in ((1, 0), (17, 3), (33, 0), (0, 5)):
        pts, bpts = parity_batch(wl, max(n, 1), nb, 0, 0.0, seed=6 + n)
        pts = pts[:n]
        L_o, g_o, res_o = N.loss_and_grad(wl, theta, pts, bpts)
        L_g, r_g, g_g, counts, _ = _run(wl, pts, bpts.reshape(-1, 3), theta)
        assert abs(L_g - L_o) <= 1e-5 * abs(L_o)
        assert rel_err(g_g, g_o) <= 1e-5


def test_cut_capacity_overflow_gives_nan():
    from paper_2210_14907_amd import NBM
    wl = I.C2
    dev = torch.device("cuda:0")
    m = NBM(wl, max_points=512, max_boundary=8, cut_capacity=4)
    pts, bpts = parity_batch(wl, 256, 8, 128, 0.01)
    p = torch.tensor(I.xavier_params(wl, 0), dtype=torch.float32, device=dev)
    tp = torch.tensor(pts, dtype=torch.float32, device=dev)
    tb = torch.tensor(bpts, dtype=torch.float32, device=dev)
    loss, _, _ = m.forward_residual(p, tp, tb)
    assert math.isnan(loss.item())
    assert m.batch_counts().cpu().numpy()[5] == 1
    # the gradient of an overflowed batch is NaN too, on the fused call and on
    # nbm_backward (which has no loss output to carry the signal)
    loss, _, grad = m.forward_residual(p, tp, tb, want_grad=True)
    assert math.isnan(loss.item()) and torch.isnan(grad).all().item()
    g2 = m.backward(p, tp, tb, dL=1.0)
    assert torch.isnan(g2).all().item()


def test_forward_residual_replays_in_a_graph():
    """forward_residual allocates nothing and records no memset, so the whole
    step (prep, forward, residuals, fused backward, reductions) can be
    captured in a HIP graph.  Every replay, with eager work of the program
    between replays, must reproduce the eager loss and gradient bit for bit."""
    from paper_2210_14907_amd import NBM
    wl = I.C2
    theta = I.xavier_params(wl, 6).astype(np.float32)
    pts, bpts = parity_batch(wl, 4096, 96, 256, 0.02, seed=9)
    m = NBM(wl, max_points=pts.shape[0], max_boundary=bpts.shape[0])
    dev = torch.device("cuda:0")
    p = torch.tensor(theta, device=dev)
    tp = torch.tensor(pts, dtype=torch.float32, device=dev)
    tb = torch.tensor(bpts, dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float64, device=dev)
    grad = torch.empty(m.P, dtype=torch.float32, device=dev)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        m.forward_residual(p, tp, tb, want_grad=True, loss=loss, grad=grad)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    loss_ref, grad_ref = loss.clone(), grad.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        m.forward_residual(p, tp, tb, want_grad=True, loss=loss, grad=grad)
    for k in range(3):
        loss.zero_()
        grad.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(loss, loss_ref) and torch.equal(grad, grad_ref), f"replay {k}"
        # eager work of the program between replays
        m.forward_residual(p * 1.01, tp, tb, want_grad=True)
        torch.cuda.synchronize()


MULTIRES_CASES = [
    # name, workload, n, nb, n_near, band
    ("c2_levels3", I.C2.replace(levels=3), 2048, 64, 256, 0.02),
    ("c3_levels2_bf16", I.C3.replace(levels=2), 1536, 48, 256, 0.01),
    ("c1_levels3", I.C1.replace(levels=3), 2048, 128, 256, 0.05),
]


@pytest.mark.parametrize("name,wl,n,nb,n_near,band", MULTIRES_CASES, ids=[c[0] for c in MULTIRES_CASES])
def test_multiresolution_step_parity(name, wl, n, nb, n_near, band):
    """Implicit refinement: every point carries cells of side h, h/2, ...,
    h/2^levels.  The GPU's summed loss and every level's residual vector
    match the oracle's; the summed gradient equals the FP64 sum of the GPU's
    single-level gradients of the same batch (the accumulation across level
    passes), and each level's gradient matches the oracle's element by
    element."""
    from tests.gpu_common import grad_block_ratios
    theta = I.xavier_params(wl, 0).astype(np.float32).astype(np.float64)
    pts, bpts = parity_batch(wl, n, nb, n_near, band, seed=13)
    pts = pts.astype(np.float32).astype(np.float64)
    bpts = bpts.astype(np.float32).astype(np.float64)
    L_o, g_o, res_o = N.loss_and_grad(wl, theta, pts, bpts)
    L_g, r_g, g_g, counts, _ = _run(wl, pts, bpts, theta, cut_capacity=pts.shape[0])
    assert counts[5] == 0 and r_g.shape == res_o["r_levels"].shape
    tol = TOL[wl.prec]
    floor = 0.1 if wl.prec == I.PREC_FP32 else 0.5
    e_loss = abs(L_g - L_o) / abs(L_o)
    per_level = (n + n_near + nb)
    e_res = max(max_rel(r_g[k * per_level:(k + 1) * per_level], res_o["r_levels"][k * per_level:(k + 1) * per_level])
                for k in range(wl.levels + 1))
    # At fine cells the boundary rows (weight 2d/h^2) dominate and the residuals'
    # signs vary, so some blocks (the biases) are sums of nearly cancelling terms:
    # entries are resolved relative to the terms' size, the oracle gradient with
    # the residuals' signs removed, summed over the levels.
    g_sum = np.zeros_like(g_g)
    scale = np.zeros_like(g_o)
    worst_level = 0.0
    for k, hl in enumerate(N.level_spacings(wl)):
        wk = wl.replace(h=hl, levels=0)
        _, g_ok, _ = N.loss_and_grad(wk, theta, pts, bpts)
        _, g_ak, _ = N.loss_and_grad(wk, theta, pts, bpts, abs_residual=True)
        sc_k = np.maximum(np.abs(g_ok), np.abs(g_ak))
        scale += sc_k
        _, _, g_k, _, _ = _run(wk, pts, bpts, theta, cut_capacity=pts.shape[0])
        g_sum += g_k.astype(np.float64)
        rk = grad_block_ratios(wk, g_k, g_ok, tol, floor, scale=sc_k)
        worst_level = max(worst_level, max(rk.values()))
        print(f"[parity] {name} level {k} (h = {hl}): worst block ratio {max(rk.values()):.3f}", flush=True)
    e_acc = rel_err(g_g, g_sum)
    ratios = grad_block_ratios(wl, g_g, g_o, tol, floor, scale=scale)
    worst = max(ratios.values())
    print(f"[parity] {name}: loss {e_loss:.2e} res (worst level) {e_res:.2e} summed-levels gradient vs sum of "
          f"single-level runs {e_acc:.2e}, block ratio {worst:.3f}, worst single level {worst_level:.3f}",
          flush=True)
    assert e_loss <= tol and e_res <= tol and worst <= 1.0 and worst_level <= 1.0
    # the levels' FP32 gradients, summed in FP64 on the device or here
    assert e_acc <= 1e-6


VARMU_CASES = [
    # the paper's convergence workload: 982-parameter sine nets (5 x 10, run
    # zero-padded to 16 wide), mu^- = y^2 ln(x+2) + 4, mu^+ = e^-z
    ("paper_5x10_varmu", I.PAPER.replace(h=1.0 / 64), 2048, 64, 256, 0.02),
    ("c2_varmu", I.C2.replace(mu_kind=I.MU_PAPER, mu_minus=4.0, mu_plus=1.0), 4096, 96, 512, 0.02),
    ("c3_varmu_bf16", I.C3.replace(mu_kind=I.MU_PAPER, mu_minus=4.0, mu_plus=1.0), 2048, 48, 256, 0.01),
]


@pytest.mark.parametrize("name,wl,n,nb,n_near,band", VARMU_CASES, ids=[c[0] for c in VARMU_CASES])
def test_variable_mu_step_parity(name, wl, n, nb, n_near, band):
    """Variable diffusion coefficients (paper Sec. 4.1): every face weighted
    by mu at its centre, jump data with mu at the projection point; loss,
    residuals and every gradient entry against the oracle (the padded
    neurons of the 10-wide nets must keep exactly zero gradients)."""
    from paper_2210_14907_amd import NBM
    from tests.gpu_common import grad_block_ratios
    theta = I.xavier_params(wl, 0).astype(np.float32).astype(np.float64)
    pts, bpts = parity_batch(wl, n, nb, n_near, band, seed=15)
    pts = pts.astype(np.float32).astype(np.float64)
    bpts = bpts.astype(np.float32).astype(np.float64)
    L_o, g_o, res_o = N.loss_and_grad(wl, theta, pts, bpts)
    dev = torch.device("cuda:0")
    m = NBM(wl, max_points=pts.shape[0], max_boundary=bpts.shape[0])
    p = m.embed(theta)
    loss, res, grad = m.forward_residual(p, torch.tensor(pts, dtype=torch.float32, device=dev),
                                         torch.tensor(bpts, dtype=torch.float32, device=dev),
                                         want_residual=True, want_grad=True)
    counts = m.batch_counts().cpu().numpy()
    torch.cuda.synchronize()
    g_all = grad.cpu().numpy().astype(np.float64)
    g_g = m.extract(grad).cpu().numpy().astype(np.float64)
    if m.padded:
        pad = np.ones(m.P, dtype=bool)
        pad[m._pad_idx] = False
        assert np.all(g_all[pad] == 0.0)
    cls = res_o["cls"]
    assert counts[2] == (cls == S.CLASS_CUT).sum() and counts[5] == 0
    tol = TOL[wl.prec]
    r_o = np.concatenate([res_o["r"], res_o["rb"]])
    e_loss, e_res = abs(loss.item() - L_o) / abs(L_o), max_rel(res.cpu().numpy(), r_o)
    ratios = grad_block_ratios(wl, g_g, g_o, tol, 0.1 if wl.prec == I.PREC_FP32 else 0.5)
    worst = max(ratios.values())
    print(f"[parity] {name}: loss {e_loss:.2e} res {e_res:.2e} grad block ratio {worst:.3f} "
          f"(cut {counts[2]})", flush=True)
    assert e_loss <= tol and e_res <= tol and worst <= 1.0
