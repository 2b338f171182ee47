"""Benchmark of the NBM training step on one MI355X.

A step is one pass of the whole hot path over one batch of synthetic input:
device sampling of the collocation points, classification, the difference-
stream MLP forward on MFMA, the cut-cell residual and FP64 loss, the fused
backward with FP64 gradient reduction, and Adam.  The batch is the 3-D sphere
workload (65,536 interior + 1,536 boundary points, two 3->64x3->1 tanh nets,
FP32 MFMA operands, h = 1/128, mu 1:10).  Inputs are resident in HBM before
the timed region.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp32": 157.3e12, "bf16": 2.5e15}

# sources the fused W=64 kernel is built from: the HBM traffic recorded in the
# counter summary applies only while they are unchanged
FUSED_SOURCES = ["nbm_fused.hip", "nbm_device.hpp", "nbm_internal.hpp", "nbm_launch.hpp"]
COUNTER_SUMMARY = os.path.join(ROOT, "profiles", "c2_k_fused_counters.md")


def kernel_source_hash():
    import hashlib
    hsh = hashlib.sha256()
    for f in FUSED_SOURCES:
        with open(os.path.join(ROOT, "paper_2210_14907_amd", "csrc", f), "rb") as fh:
            hsh.update(fh.read())
    return hsh.hexdigest()


def recorded_traffic():
    """HBM bytes per launch of the fused kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, or None when the kernel sources changed
    since those counters were taken (or no summary exists)."""
    try:
        with open(COUNTER_SUMMARY) as fh:
            text = fh.read()
    except OSError:
        return None
    vals = {}
    for ln in text.splitlines():
        ln = ln.strip().lstrip("-").strip()
        if ln.startswith(("sources_sha256:", "traffic_bytes_per_launch:")):
            k, v = ln.split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("sources_sha256") != kernel_source_hash():
        return None
    try:
        return int(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def flops_per_centre(wl):
    """Algorithmic FLOPs of evaluating one network on the 2d+1 stencil nodes
    (forward) and of the backward, per the dense layer shapes."""
    S, W, L, d = wl.n_streams, wl.width, wl.depth, wl.dim
    fwd = 2 * S * ((L - 1) * W * W + d * W + W)
    bwd = 2 * S * (2 * (L - 1) * W * W + d * W + 2 * W)
    return fwd, bwd, 2 * S * 2 * W * W   # last: one backward hidden-layer launch


def run_workload(wl, steps, warmup, seed=1, timing=True, train_to=0):
    import torch
    from paper_2210_14907_amd import NBM
    from paper_2210_14907_amd.train import init_params

    dev = torch.device("cuda:0")
    nbm = NBM(wl)
    params = init_params(wl, 0, dev)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    grad = torch.empty_like(params)
    losses = torch.empty(max(2 * steps + warmup + 64, train_to + 1) + 1, dtype=torch.float64, device=dev)
    step = 0

    def one(k):
        pts, bpts = nbm.sample_points(seed, k)
        nbm.forward_residual(params, pts, bpts, want_grad=True, loss=losses[k:k + 1], grad=grad)
        nbm.adam_step(params, m, v, grad, k, lr=wl.lr)

    for _ in range(warmup):
        step += 1
        one(step)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(steps):
        step += 1
        one(step)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    # fwd + residual + bwd only, on one resident batch
    pts, bpts = nbm.sample_points(seed, 10 ** 6)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(steps):
        nbm.forward_residual(params, pts, bpts, want_grad=True, loss=losses[0:1], grad=grad)
    ev1.record()
    torch.cuda.synchronize()
    ms_fb = ev0.elapsed_time(ev1) / steps
    # per-step distribution: each step bracketed by its own events
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(2 * steps)]
    for k in range(steps):
        step += 1
        evs[2 * k].record()
        one(step)
        evs[2 * k + 1].record()
    torch.cuda.synchronize()
    per = np.array([evs[2 * k].elapsed_time(evs[2 * k + 1]) for k in range(steps)])
    out = {"ms_per_step": ms, "ms_fwd_res_bwd": ms_fb,
           "step_ms_p10_p50_p90": [round(float(np.percentile(per, q)), 4) for q in (10, 50, 90)]}
    if timing:
        counts = nbm.batch_counts().cpu().numpy()
        nbm.set_timing(True)
        for _ in range(max(3, min(steps, 20))):
            step += 1
            one(step)
        tm = nbm.read_timing()
        nbm.set_timing(False)
        counts = nbm.batch_counts().cpu().numpy()
        out["timing"] = tm
        out["counts"] = counts
    if train_to > step:
        while step < train_to:
            step += 1
            one(step)
        torch.cuda.synchronize()
    out["steps_trained"] = step
    out["final_loss"] = float(losses[step].item())
    out["params"] = params
    out["nbm"] = nbm
    return out


def accuracy(wl, res, judge_n, judge=None):
    """L-inf / L2 of the trained surrogate at the interior nodes of a judge
    grid, against the closed-form solution and the FP64 grid CG oracle.
    `judge` = (GridSystem, solution, seconds) reuses an earlier solve."""
    import torch
    from oracle import grid as OG

    nbm, params = res["nbm"], res["params"]
    if judge is None:
        gs = OG.GridSystem(wl, judge_n)
        t0 = time.time()
        U = gs.solve()
        t_judge = time.time() - t0
    else:
        gs, U, t_judge = judge
    res["judge"] = (gs, U, t_judge)
    xin = gs.x[gs.interior]
    q = torch.tensor(xin, dtype=torch.float32, device=nbm.device)
    u = np.concatenate([nbm.eval(params, q[i:i + 60000]).cpu().numpy() for i in range(0, len(q), 60000)])
    out = {"judge_n": judge_n, "judge_seconds": round(t_judge, 2)}
    e = u - U[gs.interior]
    out["linf_vs_grid"] = float(np.abs(e).max())
    out["l2_vs_grid"] = float(np.sqrt(np.mean(e * e)))
    if gs.prob.has_exact():
        ex = gs.prob.u_exact(xin)
        out["linf_vs_exact"] = float(np.abs(u - ex).max())
        out["l2_vs_exact"] = float(np.sqrt(np.mean((u - ex) ** 2)))
        out["grid_linf_vs_exact"] = float(np.abs(U[gs.interior] - ex).max())
    return out


def cpu_baseline(wl, target_s=12.0):
    """The FP64 oracle's step (point evaluation + reverse mode) on a bounded
    sample of the same workload, timed on the host cores: batches of up to
    the workload's size, repeated until about target_s seconds of work."""
    from threadpoolctl import threadpool_info

    import nbm_inputs as I
    from oracle import nbm as ON

    theta = I.xavier_params(wl, 0)
    n0 = 2048
    pts, bpts = I.collocation_batch(wl, n0, max(1, int(round(n0 * wl.dim * wl.h))), seed=11)
    t = time.time()
    ON.loss_and_grad(wl, theta, pts, bpts)
    rate0 = n0 / (time.time() - t)
    n = int(min(wl.n_points, max(n0, rate0 * target_s)))
    nb = int(round(n * wl.dim * wl.h))
    reps = max(1, min(64, int(target_s * rate0 / n)))
    dt, done = 0.0, 0
    for k in range(reps):
        pts, bpts = I.collocation_batch(wl, n, nb, seed=12 + k)
        t = time.time()
        ON.loss_and_grad(wl, theta, pts, bpts)
        dt += time.time() - t
        done += n
        if dt >= target_s:
            break
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    # one thread, on a smaller batch
    from threadpoolctl import threadpool_limits
    n1 = 4096
    pts1, bpts1 = I.collocation_batch(wl, n1, int(round(n1 * wl.dim * wl.h)), seed=40)
    with threadpool_limits(limits=1):
        t = time.time()
        ON.loss_and_grad(wl, theta, pts1, bpts1)
        dt1 = time.time() - t
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": round(done / dt, 1), "unit": "colloc pts/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{done // n} batch(es) of {n} interior + {nb} boundary points of the same workload, "
                      f"one FP64 step (loss + gradient) each, {dt:.1f} s",
            "single_thread_value": round(n1 / dt1, 1), "cpu_model": model, "host_cpus": os.cpu_count()}


def eval_rate(tiles=6, warm=2):
    """Evaluation throughput of the 1024^3 grid workload: the star-interface
    networks (3 -> 128x4 -> 1 sin, BF16 MFMA operands) on 2^24-point tiles of the
    grid, coordinates generated in-kernel.  Per query: 2*3*128 (layer 1) +
    3*2*128^2 (hidden layers) + 2*128 (output) = 99,328 FLOP, 98,304 of them on MFMA."""
    import torch
    import nbm_inputs as I
    from paper_2210_14907_amd.binding import NBM
    wl, m, gn = I.C4, 1 << 24, 1024
    nbm = NBM(wl, max_points=m, max_boundary=0, eval_only=True)
    params = torch.tensor(I.xavier_params(wl, 0), dtype=torch.float32, device=nbm.device)
    out = torch.empty(m, dtype=torch.float32, device=nbm.device)
    for k in range(warm):
        nbm.eval(params, m=m, tile_index=k, grid_n=gn, out=out)
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for k in range(tiles):
        nbm.eval(params, m=m, tile_index=warm + k, grid_n=gn, out=out)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / tiles
    flop_q, mfma_q = 99328, 98304
    del nbm, out
    torch.cuda.empty_cache()
    return {"workload": "c5_grid1024_eval (star networks 3->128x4->1 sin, BF16, 2^24-point tiles)",
            "tile_points": m, "ms_per_tile": round(ms, 4), "pts_per_s": round(m / (ms * 1e-3), 1),
            "grid_1024_cubed_s": round(ms * 64 * 1e-3, 4), "flop_per_query": flop_q,
            "tflops": round(flop_q * m / (ms * 1e-3) / 1e12, 2),
            "mfma_frac_bf16_peak": round(mfma_q * m / (ms * 1e-3) / PEAK["bf16"], 4)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--workload", default="c2", help="c2 (default, the headline line) or c1/c3/c4 for profiling")
    ap.add_argument("--prec", choices=("fp32", "bf16"), default=None,
                    help="operand precision of the workload, for profiling (default: the workload's own)")
    ap.add_argument("--only-eval", action="store_true",
                    help="print only the evaluation throughput of the 1024^3 grid workload (profiling)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="run one device copy of this many MiB first (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU (data-parallel) path.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import nbm_inputs as I

    if args.only_eval:
        print(json.dumps({"eval_c5": eval_rate()}), flush=True)
        return
    wl = I.WORKLOADS[args.workload]
    if args.prec:
        prec = I.PREC_BF16 if args.prec == "bf16" else I.PREC_FP32
        if prec != wl.prec:
            wl = wl.replace(prec=prec, name=wl.name.rsplit("_", 1)[0] + "_" + args.prec)
    if args.calib_copy_mb:
        nbytes = args.calib_copy_mb << 20
        a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    res = run_workload(wl, args.steps, args.warmup, train_to=0 if args.no_accuracy else wl.steps)
    n_step = wl.n_points
    value = n_step / (res["ms_per_step"] * 1e-3)
    fwd_f, bwd_f, bl_f = flops_per_centre(wl)
    tm = res["timing"]
    c = res["counts"]
    nbr = 2 * wl.dim if wl.mu_minus != wl.mu_plus else 0
    centres = int(c[0] + c[1] + (2 + nbr) * c[2] + c[3] + c[4])
    f_ms, f_n = tm["forward"]
    b_ms, b_n = tm["backward"]
    if wl.width == 64:
        # one launch per step runs the forward, residual and backward of every
        # tile on chip; it is the dominant kernel
        name, per_launch, avg = ("k_fused (forward + residual + backward, all layers)",
                                 (fwd_f + bwd_f) * centres, b_ms / b_n)
    elif b_ms >= f_ms:
        name, per_launch, avg = "backward group", bwd_f * centres, b_ms / b_n
    else:
        name, per_launch, avg = "k_forward (all layers)", fwd_f * centres, f_ms / f_n
    dtype = "fp32" if wl.prec == I.PREC_FP32 else "bf16"
    achieved = per_launch / (avg * 1e-3)
    line = {
        "metric": "colloc pts/s (fwd+FV residual+bwd), BF16 vs FP32, at stated Linf vs FP64 oracle",
        "value": round(value, 1),
        "unit": "colloc pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["ms_per_step"], 4),
        "step_ms_p10_p50_p90": res["step_ms_p10_p50_p90"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if wl.prec == I.PREC_FP32 else "bf16",
        "data": "synthetic (Philox lattice points, manufactured sphere solution, Xavier init seed 0)",
        "config": {"workload": wl.name, "n_points": wl.n_points, "n_boundary": wl.n_boundary,
                   "h": wl.h, "net": f"2 x {wl.dim}->{wl.width}x{wl.depth}->1 {'tanh' if wl.act == I.ACT_TANH else 'sin'}",
                   "mu": [wl.mu_minus, wl.mu_plus]},
        "fwd_res_bwd_pts_per_s": round(n_step / (res["ms_fwd_res_bwd"] * 1e-3), 1),
        "kernel_ms_per_step": {k: round(v[0] / max(1, tm["forward"][1]), 4) for k, v in tm.items() if v[1]},
        "roofline": {"bound": "mfma", "kernel": name, "achieved": achieved / 1e12,
                     "peak": PEAK[dtype] / 1e12, "unit": "TFLOP/s", "frac": achieved / PEAK[dtype],
                     "traffic": recorded_traffic() if wl.width == 64 and wl.prec == I.PREC_FP32 else None,
                     "flop_per_launch": per_launch, "avg_launch_ms": avg},
    }
    if not args.no_accuracy and wl.problem != I.PROB_FOURIER:
        acc = accuracy(wl, res, 64)
        acc["steps_trained"] = res["steps_trained"]
        acc["final_loss"] = res["final_loss"]
        line["accuracy"] = acc
        if wl.prec == I.PREC_FP32:
            # the same training in BF16 operands, judged on the same grid solution
            wb = wl.replace(prec=I.PREC_BF16)
            rb = run_workload(wb, 10, 3, timing=False, train_to=wb.steps)
            ab = accuracy(wb, rb, 64, judge=res["judge"])
            ab["steps_trained"] = rb["steps_trained"]
            ab["final_loss"] = rb["final_loss"]
            ab["linf_ratio_bf16_over_fp32"] = ab["linf_vs_grid"] / acc["linf_vs_grid"]
            line["accuracy_bf16"] = ab
            del rb
            torch.cuda.empty_cache()
    if not args.no_extra:
        extra = {}
        for tag, w in (("c2_bf16", wl.replace(prec=I.PREC_BF16)), ("c3_bf16", I.C3),
                       ("c3_fp32", I.C3.replace(prec=I.PREC_FP32)), ("c4_bf16", I.C4)):
            r = run_workload(w, max(10, args.steps // 2), 3, timing=False)
            extra[tag] = {"pts_per_s": round(w.n_points / (r["ms_per_step"] * 1e-3), 1),
                          "fwd_res_bwd_pts_per_s": round(w.n_points / (r["ms_fwd_res_bwd"] * 1e-3), 1),
                          "ms_per_step": round(r["ms_per_step"], 4)}
            del r
            torch.cuda.empty_cache()
        line["same_step_other_precisions"] = extra
        line["eval_c5"] = eval_rate()
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
