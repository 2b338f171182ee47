"""Thin ctypes binding of libnbm.so (argument marshalling only).

Every step of the NBM path runs in the library's gfx950 kernels; PyTorch only
provides device memory and the current HIP stream.  Loading fails loudly if
the library has not been built.
"""
from __future__ import annotations

import ctypes
from pathlib import Path

import numpy as np
import torch

import nbm_inputs as I

LIB_PATH = Path(__file__).resolve().parent / "libnbm.so"
_lib = None

EXPORTS = ["nbm_create", "nbm_destroy", "nbm_param_count", "nbm_workspace_bytes", "nbm_prepare",
           "nbm_sample_points", "nbm_forward_residual", "nbm_forward_residual_noalloc", "nbm_backward", "nbm_adam_step", "nbm_eval",
           "nbm_grid_interp",
           "nbm_batch_counts", "nbm_set_timing", "nbm_read_timing", "nbm_last_error"]


class NbmConfig(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("width", ctypes.c_int32), ("depth", ctypes.c_int32),
                ("act", ctypes.c_int32), ("prec", ctypes.c_int32), ("h", ctypes.c_double),
                ("interface_kind", ctypes.c_int32), ("radius", ctypes.c_double),
                ("star_amp", ctypes.c_double), ("plane_n", ctypes.c_double * 3),
                ("plane_c", ctypes.c_double), ("mu_minus", ctypes.c_double),
                ("mu_plus", ctypes.c_double), ("mu_kind", ctypes.c_int32), ("k_minus", ctypes.c_double),
                ("k_plus", ctypes.c_double), ("problem", ctypes.c_int32),
                ("alpha_const", ctypes.c_double), ("beta_const", ctypes.c_double),
                ("lin_a", ctypes.c_double * 4), ("lin_b", ctypes.c_double * 4),
                ("n_modes", ctypes.c_int32), ("mode_k", ctypes.POINTER(ctypes.c_int32)),
                ("mode_a", ctypes.POINTER(ctypes.c_double)), ("mode_b", ctypes.POINTER(ctypes.c_double)),
                ("max_points", ctypes.c_int64), ("max_boundary", ctypes.c_int64),
                ("cut_capacity", ctypes.c_int64), ("eval_only", ctypes.c_int32),
                ("phi_n", ctypes.c_int32), ("phi_table", ctypes.POINTER(ctypes.c_double)),
                ("levels", ctypes.c_int32)]


class NbmError(RuntimeError):
    pass


# hidden widths with compiled kernels; narrower networks run zero-padded to
# the next one (padded neurons have zero weights in and out, so their
# pre-activations, activations and gradients are exactly zero)
COMPILED_WIDTHS = (16, 64, 128)


def device_width(width: int) -> int:
    for w in COMPILED_WIDTHS:
        if width <= w:
            return w if (width == w or w == 16) else width
    return width


def _param_blocks(width, dim, depth):
    """(rows, cols) of every parameter block of one net, in packing order."""
    blocks = [(width, dim), (width, 1)]
    for _ in range(depth - 1):
        blocks += [(width, width), (width, 1)]
    blocks += [(1, width), (1, 1)]
    return blocks


def padding_index(wl: I.Workload, wdev: int) -> np.ndarray:
    """Positions in the width-wdev parameter vector of the wl.width one's
    entries (both nets, packing order)."""
    small = _param_blocks(wl.width, wl.dim, wl.depth)
    big = _param_blocks(wdev, wl.dim, wl.depth)
    idx, off = [], 0
    for _net in range(2):
        for (r, c), (R, C) in zip(small, big):
            rr, cc = np.meshgrid(np.arange(r), np.arange(c), indexing="ij")
            idx.append((off + rr * C + cc).ravel())
            off += R * C
    return np.concatenate(idx)


def lib():
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise NbmError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(there is no CPU fallback)")
        L = ctypes.CDLL(str(LIB_PATH))
        vp, i64, f32, f64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_float, ctypes.c_double
        L.nbm_create.argtypes = [ctypes.POINTER(NbmConfig), ctypes.POINTER(vp)]
        L.nbm_destroy.argtypes = [vp]
        L.nbm_destroy.restype = None
        L.nbm_param_count.argtypes = [vp]
        L.nbm_param_count.restype = i64
        L.nbm_workspace_bytes.argtypes = [vp, i64, i64]
        L.nbm_workspace_bytes.restype = ctypes.c_size_t
        L.nbm_prepare.argtypes = [vp, vp, vp, ctypes.c_size_t]
        L.nbm_sample_points.argtypes = [vp, vp, ctypes.c_uint64, i64, vp, i64, vp, i64]
        L.nbm_forward_residual.argtypes = [vp, vp, vp, vp, i64, vp, i64, vp, vp, vp, vp, ctypes.c_size_t]
        L.nbm_forward_residual_noalloc.argtypes = [vp, vp, vp, vp, i64, vp, i64, vp, vp, vp]
        L.nbm_backward.argtypes = [vp, vp, vp, vp, i64, vp, i64, f64, vp, vp, ctypes.c_size_t]
        L.nbm_adam_step.argtypes = [vp, vp, vp, vp, vp, vp, i64, f32, f32, f32, f32]
        L.nbm_eval.argtypes = [vp, vp, vp, vp, i64, i64, ctypes.c_int32, vp, vp, ctypes.c_size_t]
        L.nbm_grid_interp.argtypes = [vp, vp, vp, ctypes.c_int32, i64, ctypes.c_int32, i64, vp]
        L.nbm_batch_counts.argtypes = [vp, vp, vp, vp, ctypes.c_size_t]
        L.nbm_set_timing.argtypes = [vp, ctypes.c_int]
        L.nbm_read_timing.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
        L.nbm_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise NbmError(f"nbm error {rc}: {lib().nbm_last_error().decode()}")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class NBM:
    """One NBM problem/network configuration with its device workspace."""

    def __init__(self, wl: I.Workload, max_points: int = None, max_boundary: int = None,
                 cut_capacity: int = 0, device: str = "cuda:0", eval_only: bool = False):
        self.wl = wl
        self.device = torch.device(device)
        # narrower networks run zero-padded to a compiled width: the parameter
        # vectors of every call are then the padded ones (embed / extract)
        wdev = device_width(wl.width)
        self.padded = wdev != wl.width
        self._pad_idx = padding_index(wl, wdev) if self.padded else None
        wl = wl.replace(width=wdev) if self.padded else wl
        cfg = NbmConfig()
        cfg.dim, cfg.width, cfg.depth = wl.dim, wl.width, wl.depth
        cfg.act, cfg.prec, cfg.h = wl.act, wl.prec, wl.h
        cfg.interface_kind, cfg.radius, cfg.star_amp = wl.interface, wl.radius, wl.star_amp
        for i in range(3):
            cfg.plane_n[i] = wl.plane_n[i]
        cfg.plane_c = wl.plane_c
        cfg.mu_minus, cfg.mu_plus = wl.mu_minus, wl.mu_plus
        cfg.mu_kind = wl.mu_kind
        cfg.k_minus, cfg.k_plus = wl.k_minus, wl.k_plus
        cfg.problem = wl.problem
        cfg.alpha_const, cfg.beta_const = wl.alpha_const, wl.beta_const
        for i in range(4):
            cfg.lin_a[i], cfg.lin_b[i] = wl.lin_a[i], wl.lin_b[i]
        if wl.problem == I.PROB_FOURIER:
            k, a, b = I.fourier_modes(wl)
            self._k = np.ascontiguousarray(k, dtype=np.int32)
            self._a = np.ascontiguousarray(a, dtype=np.float64)
            self._b = np.ascontiguousarray(b, dtype=np.float64)
            cfg.n_modes = len(k)
            cfg.mode_k = self._k.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            cfg.mode_a = self._a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            cfg.mode_b = self._b.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        cfg.max_points = wl.n_points if max_points is None else max_points
        cfg.max_boundary = wl.n_boundary if max_boundary is None else max_boundary
        cfg.cut_capacity = cut_capacity
        cfg.eval_only = 1 if eval_only else 0
        cfg.levels = wl.levels
        if wl.interface == I.IFACE_GRID:
            self._phitab = np.ascontiguousarray(I.phi_table(wl), dtype=np.float64)
            cfg.phi_n = wl.phi_n
            cfg.phi_table = self._phitab.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self.cfg = cfg
        h = ctypes.c_void_p()
        _check(lib().nbm_create(ctypes.byref(cfg), ctypes.byref(h)))
        self.ctx = h
        self.P = lib().nbm_param_count(h)
        self.ws_bytes = lib().nbm_workspace_bytes(h, cfg.max_points, 0 if eval_only else cfg.max_boundary)
        if self.ws_bytes == 0:
            raise NbmError("nbm_workspace_bytes rejected the batch capacity")
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.ws.data_ptr()) % 256
        self.ws_view = self.ws[off:off + self.ws_bytes]
        with torch.cuda.device(self.device):
            _check(lib().nbm_prepare(h, _stream(), _ptr(self.ws_view), self.ws_bytes))

    def embed(self, theta):
        """Parameters of the workload's own width -> the device parameter
        vector (zero-padded when the width is not compiled).  numpy or torch
        in, FP32 device tensor out."""
        t = torch.as_tensor(np.asarray(theta) if not torch.is_tensor(theta) else theta)
        t = t.to(device=self.device, dtype=torch.float32)
        if not self.padded:
            return t.clone()
        out = torch.zeros(self.P, dtype=torch.float32, device=self.device)
        out[torch.from_numpy(self._pad_idx).to(self.device)] = t
        return out

    def extract(self, vec):
        """Device parameter-sized vector -> the entries of the workload's own width."""
        if not self.padded:
            return vec
        return vec[torch.from_numpy(self._pad_idx).to(vec.device)]

    def __del__(self):
        try:
            if getattr(self, "ctx", None):
                lib().nbm_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass

    # -- entry points --------------------------------------------------------
    def sample_points(self, seed: int, step: int, n: int = None, nb: int = None):
        n = self.wl.n_points if n is None else n
        nb = self.wl.n_boundary if nb is None else nb
        pts = torch.empty((n, self.wl.dim), dtype=torch.float32, device=self.device)
        bpts = torch.empty((nb, self.wl.dim), dtype=torch.float32, device=self.device)
        _check(lib().nbm_sample_points(self.ctx, _stream(), seed, step, _ptr(pts), n, _ptr(bpts), nb))
        return pts, bpts

    def forward_residual(self, params, pts, bpts, want_residual=False, want_grad=False,
                         loss=None, grad=None, residual=None):
        n, nb = pts.shape[0], bpts.shape[0]
        if loss is None:
            loss = torch.empty(1, dtype=torch.float64, device=self.device)
        if want_residual and residual is None:
            residual = torch.empty((self.wl.levels + 1) * (n + nb), dtype=torch.float32, device=self.device)
        if want_grad and grad is None:
            grad = torch.empty(self.P, dtype=torch.float32, device=self.device)
        _check(lib().nbm_forward_residual(self.ctx, _stream(), _ptr(params), _ptr(pts), n, _ptr(bpts), nb,
                                          _ptr(residual) if want_residual else None, _ptr(loss),
                                          _ptr(grad) if want_grad else None, _ptr(self.ws_view),
                                          self.ws_bytes))
        return loss, (residual if want_residual else None), (grad if want_grad else None)

    def forward_residual_noalloc(self, params, pts, bpts, loss, residual=None, grad=None):
        """nbm_forward_residual_noalloc: the same step in the library's static
        per-GPU scratch (no workspace); every output buffer is the caller's."""
        _check(lib().nbm_forward_residual_noalloc(self.ctx, _stream(), _ptr(params), _ptr(pts), pts.shape[0],
                                                  _ptr(bpts), bpts.shape[0], _ptr(residual), _ptr(loss),
                                                  _ptr(grad)))
        return loss, residual, grad

    def backward(self, params, pts, bpts, dL=1.0, grad=None):
        if grad is None:
            grad = torch.empty(self.P, dtype=torch.float32, device=self.device)
        _check(lib().nbm_backward(self.ctx, _stream(), _ptr(params), _ptr(pts), pts.shape[0], _ptr(bpts),
                                  bpts.shape[0], float(dL), _ptr(grad), _ptr(self.ws_view), self.ws_bytes))
        return grad

    def adam_step(self, params, m, v, grad, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        _check(lib().nbm_adam_step(self.ctx, _stream(), _ptr(params), _ptr(m), _ptr(v), _ptr(grad),
                                   int(step), lr, beta1, beta2, eps))

    def eval(self, params, query=None, m=None, tile_index=0, grid_n=0, out=None):
        """u at query points [m][d] (split into calls of at most max_points),
        or at grid tile `tile_index` of m points of the grid_n^d lattice."""
        if query is not None:
            m = query.shape[0]
        if out is None:
            out = torch.empty(m, dtype=torch.float32, device=self.device)
        cap = int(self.cfg.max_points)
        if query is None:
            _check(lib().nbm_eval(self.ctx, _stream(), _ptr(params), None, m, tile_index, grid_n,
                                  _ptr(out), _ptr(self.ws_view), self.ws_bytes))
            return out
        for i in range(0, m, cap):
            q = query[i:i + cap]
            o = out[i:i + cap]
            _check(lib().nbm_eval(self.ctx, _stream(), _ptr(params), _ptr(q), q.shape[0], 0, 0,
                                  _ptr(o), _ptr(self.ws_view), self.ws_bytes))
        return out

    def grid_interp(self, U, judge_n, tile_index, grid_n, m, out=None):
        """Multilinear interpolation of the nodal FP64 device array U
        [(judge_n+1)^d] at tile `tile_index` of m points of the grid_n^d lattice."""
        if out is None:
            out = torch.empty(m, dtype=torch.float32, device=self.device)
        if U.dtype != torch.float64 or U.numel() != (judge_n + 1) ** self.wl.dim:
            raise NbmError("U must be a float64 array of (judge_n + 1)^d nodal values")
        _check(lib().nbm_grid_interp(self.ctx, _stream(), _ptr(U), int(judge_n), int(tile_index), int(grid_n),
                                     int(m), _ptr(out)))
        return out

    TIMING_GROUPS = ["prep", "forward", "residual", "backward", "reduce", "adam", "sample", "eval",
                     "weight_grad", "forcing"]

    def set_timing(self, enable: bool):
        _check(lib().nbm_set_timing(self.ctx, 1 if enable else 0))

    def read_timing(self):
        """{group: (total ms, launches)} since the last read (blocks the host)."""
        ng = len(self.TIMING_GROUPS)
        ms = (ctypes.c_double * ng)()
        n = (ctypes.c_int64 * ng)()
        _check(lib().nbm_read_timing(self.ctx, ms, n))
        return {g: (ms[i], n[i]) for i, g in enumerate(self.TIMING_GROUPS)}

    def batch_counts(self):
        c = torch.zeros(8, dtype=torch.int32, device=self.device)
        _check(lib().nbm_batch_counts(self.ctx, _stream(), _ptr(c), _ptr(self.ws_view), self.ws_bytes))
        return c
