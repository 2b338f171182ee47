"""Training on the GPU through the C ABI (paper Sec. 3: the networks are
adjusted by Adam using gradients of the aggregated residual loss).

`NBMResidual` is the torch.autograd.Function wrapper of the fused forward +
residual + backward call: because the loss is the terminal scalar, its
backward returns the fused gradient times the upstream gradient.  `train`
runs the step loop entirely on the device (sampling, fused step, Adam) and
reads the loss history back once at the end.
"""
from __future__ import annotations

import torch

import nbm_inputs as I
from .binding import NBM


class NBMResidual(torch.autograd.Function):
    """loss = NBMResidual.apply(params, pts, bpts, nbm, fused=True).

    fused=True: the forward call also writes dL/dtheta (one fused pass), the
    backward returns it times the upstream gradient.  fused=False: the
    forward computes only the loss, the backward calls nbm_backward with the
    upstream gradient as its factor (the step is recomputed; nothing is
    stored between the two calls)."""

    @staticmethod
    def forward(ctx, params, pts, bpts, nbm: NBM, fused: bool = True):
        p = params.detach()
        if fused:
            loss, _, grad = nbm.forward_residual(p, pts, bpts, want_grad=True)
            ctx.save_for_backward(grad)
        else:
            loss, _, _ = nbm.forward_residual(p, pts, bpts)
            ctx.save_for_backward(p, pts, bpts)
        ctx.nbm, ctx.fused = nbm, fused
        return loss.reshape(())

    @staticmethod
    def backward(ctx, gout):
        if ctx.fused:
            (grad,) = ctx.saved_tensors
            return grad * gout.to(grad.dtype), None, None, None, None
        p, pts, bpts = ctx.saved_tensors
        grad = ctx.nbm.backward(p, pts, bpts, dL=float(gout.item()))
        return grad, None, None, None, None


def nbm_loss(params, pts, bpts, nbm: NBM, fused: bool = True):
    return NBMResidual.apply(params, pts, bpts, nbm, fused)


def init_params(wl: I.Workload, seed: int = 0, device="cuda:0"):
    return torch.tensor(I.xavier_params(wl, seed), dtype=torch.float32, device=device)


def train(wl: I.Workload, steps: int = None, lr: float = None, seed: int = 1, params=None,
          nbm: NBM = None, start_step: int = 1, state=None, log_every: int = 0,
          check_finite: bool = True):
    """Adam training loop; returns (params, nbm, state, losses[cpu float64])."""
    steps = wl.steps if steps is None else steps
    lr = wl.lr if lr is None else lr
    nbm = NBM(wl) if nbm is None else nbm
    dev = nbm.device
    params = nbm.embed(I.xavier_params(wl, 0)) if params is None else params
    if state is None:
        state = {"m": torch.zeros_like(params), "v": torch.zeros_like(params)}
    losses = torch.empty(steps, dtype=torch.float64, device=dev)
    grad = torch.empty_like(params)
    for k in range(steps):
        step = start_step + k
        pts, bpts = nbm.sample_points(seed, step)
        nbm.forward_residual(params, pts, bpts, want_grad=True, loss=losses[k:k + 1], grad=grad)
        nbm.adam_step(params, state["m"], state["v"], grad, step, lr=lr)
        if log_every and (k + 1) % log_every == 0:
            print(f"step {step}: loss {losses[k].item():.6e}", flush=True)
    losses = losses.cpu()
    if check_finite and not torch.isfinite(losses).all():
        bad = int((~torch.isfinite(losses)).nonzero()[0, 0]) + start_step
        raise RuntimeError(f"non-finite loss at step {bad} (a batch over the cut capacity "
                           "reports NaN loss and gradient)")
    return params, nbm, state, losses
