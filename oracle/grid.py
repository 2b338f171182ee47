"""Grid judge: the cut-cell scheme assembled on a uniform grid and solved by
PCG in FP64 (oracle).

Grid with n intervals per axis on [-1,1]^d, spacing h = 2/n, unknowns at the
interior nodes, Dirichlet nodes held at g.  Every interior node carries the
row R_p = 0 of the cell residual (same geometry and jump extension as the
collocation residual), written as

    sum_F c_F (U_p - U_F) + h^2 kap_p U_p = -h^2 K_p,   kap_p = sum_s k^s v^s,

which is symmetric because c_F depends only on the face.  With a coefficient
contrast, the jump extension needs the normal derivative of the low-mu side;
it is lagged (Picard iteration): after each solve the low-mu field is extended
across Gamma by upwind PDE extrapolation along the normal (constant normal
derivative), its central-difference gradient is taken at the cut-cell nodes,
and the right-hand side is rebuilt.  The iteration is accelerated with
Anderson mixing on the lagged gradients.
"""
from __future__ import annotations

import ctypes
import hashlib
import os
import tempfile
from pathlib import Path

import numpy as np

import nbm_inputs as I
from . import geometry as G
from . import scheme as S
from .problems import Problem

_HERE = Path(__file__).resolve().parent
_LIB = None


def build_solver() -> Path:
    so = _HERE / "_grid_solver.so"
    src = _HERE / "grid_solver.c"
    if (not so.exists()) or so.stat().st_mtime < src.stat().st_mtime:
        import subprocess
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-o", str(so), str(src)])
    return so


def _lib():
    global _LIB
    if _LIB is None:
        _LIB = ctypes.CDLL(str(build_solver()))
        dp = ctypes.POINTER(ctypes.c_double)
        _LIB.nbm_oracle_pcg.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, dp, ctypes.c_double,
                                        ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int), dp]
        _LIB.nbm_oracle_apply.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, dp]
    return _LIB


def _ptr(a):
    if a is None:
        return ctypes.POINTER(ctypes.c_double)()
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def pcg(d, n, cface, b, u0=None, tol=1e-12, maxit=5000, precond="mg", kdiag=None):
    cface = np.ascontiguousarray(cface, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64).ravel()
    kd = None if kdiag is None else np.ascontiguousarray(kdiag, dtype=np.float64)
    u = np.zeros_like(b) if u0 is None else np.ascontiguousarray(u0, dtype=np.float64).ravel().copy()
    it = ctypes.c_int(0)
    rr = ctypes.c_double(0)
    rc = _lib().nbm_oracle_pcg(d, n, _ptr(cface), _ptr(kd), _ptr(b), _ptr(u), tol, maxit,
                               1 if precond == "mg" else 0, ctypes.byref(it), ctypes.byref(rr))
    if rc != 0:
        raise RuntimeError("pcg failed")
    return u, it.value, rr.value


def apply_A(d, n, cface, u, kdiag=None):
    cface = np.ascontiguousarray(cface, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64).ravel()
    kd = None if kdiag is None else np.ascontiguousarray(kdiag, dtype=np.float64)
    y = np.zeros_like(u)
    _lib().nbm_oracle_apply(d, n, _ptr(cface), _ptr(kd), _ptr(u), _ptr(y))
    return y


class PicardNotConverged(RuntimeError):
    """The lagged low-mu gradient iteration missed its tolerance."""


class GridSystem:
    """Assembled grid rows for one workload at n intervals per axis.

    Arrays are stored on all (n+1)^d nodes in C order with axis 0 fastest
    (flat index = i0 + (n+1) i1 + (n+1)^2 i2)."""

    def __init__(self, wl: I.Workload, n: int):
        self.wl, self.n, self.d = wl, n, wl.dim
        self.h = 2.0 / n
        self.prob = Problem(wl)
        d, h = self.d, self.h
        ax = -1.0 + h * np.arange(n + 1)
        mesh = np.meshgrid(*([ax] * d), indexing="ij")
        # flat order with axis 0 fastest: transpose the ij grid
        self.x = np.stack([m.transpose().ravel() for m in mesh], axis=-1)
        self.shape = (n + 1,) * d
        self.N = self.x.shape[0]
        idx = np.stack(np.unravel_index(np.arange(self.N), self.shape[::-1]), axis=-1)[:, ::-1]
        self.idx = idx
        self.interior = np.all((idx > 0) & (idx < n), axis=1)
        self.stride = np.array([(n + 1) ** a for a in range(d)])
        self.side = G.side_minus(wl, self.x)
        # dual grid of cell corners: -1 - h/2 + k h, k = 0..n+1
        axd = -1.0 - 0.5 * h + h * np.arange(n + 2)
        md = np.meshgrid(*([axd] * d), indexing="ij")
        xd = np.stack([m.transpose().ravel() for m in md], axis=-1)
        self.phid = G.phi(wl, xd).reshape((n + 2,) * d)       # indexed [i_{d-1}, ..., i_0]
        self.sided = G.side_minus(wl, xd).reshape((n + 2,) * d)
        self._faces()
        self._classify()

    # node p (idx i) has cell corners at dual indices i + {0,1}^d
    def _faces(self):
        d, n = self.d, self.n
        cface = np.zeros((d, self.N))
        phid = self.phid
        for a in range(d):
            # face between node i and i + e_a: dual corners with index i_a + 1 along a,
            # i_b + {0, 1} across.
            fr = np.zeros(self.N)
            ii = self.idx
            ok = ii[:, a] < n
            sel = np.nonzero(ok)[0]
            others = [b for b in range(d) if b != a]
            corner_vals = []
            for m in range(1 << (d - 1)):
                j = ii[sel].copy()
                j[:, a] += 1
                for t, b in enumerate(others):
                    j[:, b] += (m >> t) & 1
                corner_vals.append(phid[tuple(j[:, k] for k in range(d - 1, -1, -1))])
            fv = np.stack(corner_vals, axis=-1)
            sides = fv < 0
            mixed = sides.any(axis=1) & ~sides.all(axis=1)
            val = np.where(sides.all(axis=1), 1.0, 0.0)
            if mixed.any():
                fm = fv[mixed]
                if d == 2:
                    val[mixed] = G.seg_neg_fraction(fm[:, 0], fm[:, 1])
                else:
                    val[mixed] = 0.5 * (G.tri_neg_fraction(fm[:, [0, 1, 3]]) +
                                        G.tri_neg_fraction(fm[:, [0, 2, 3]]))
            fr[sel] = val
            # mu^s at the face centre x_p + (h/2) e_a
            xf = self.x.copy()
            xf[:, a] += 0.5 * self.h
            mm, mp = self.prob.mu_at(0, xf), self.prob.mu_at(1, xf)
            cface[a] = np.where(ok, mm * fr + mp * (1.0 - fr), 0.0)
        self.cface = cface

    def _classify(self):
        d, n = self.d, self.n
        ip = np.nonzero(self.interior)[0]
        ii = self.idx[ip]
        s0 = self.side[ip]
        same = np.ones(ip.size, dtype=bool)
        for a in range(d):
            for sgn in (1, -1):
                same &= self.side[ip + sgn * self.stride[a]] == s0
        for m in range(1 << d):
            j = ii + np.array([(m >> a) & 1 for a in range(d)])
            same &= self.sided[tuple(j[:, k] for k in range(d - 1, -1, -1))] == s0
        self.cut = ip[~same]
        self.uncut = ip[same]

    def node_offsets(self):
        d = self.d
        off = [0]
        for a in range(d):
            off += [self.stride[a], -self.stride[a]]
        return np.array(off)

    def rhs(self, grad_lo_cut=None):
        """-h^2 K at every interior node (+ Dirichlet data of boundary
        neighbours).  grad_lo_cut[ncut, 2d+1, d]: lagged low-mu gradients at
        the nodes of the cut cells (contrast only)."""
        d, h, wl, prob = self.d, self.h, self.wl, self.prob
        b = np.zeros(self.N)
        if not hasattr(self, "_f_uncut"):
            # everything but the lagged gradients is the same in every Picard
            # iteration: forcing, cut-cell geometry, interface data at the nodes
            if wl.problem == I.PROB_FOURIER:
                fn = prob.f_grid(self.n)               # f^- = f^+ at every node
                fcut = (fn[self.cut], fn[self.cut])
                self._f_uncut = fn[self.uncut]
                del fn
            else:
                xu = self.x[self.uncut]
                su = self.side[self.uncut]
                self._f_uncut = np.where(su, prob.f_side(0, xu), prob.f_side(1, xu))
                xc = self.x[self.cut]
                fcut = (prob.f_side(0, xc), prob.f_side(1, xc))
            if self.cut.size:
                nodes = self.cut[:, None] + self.node_offsets()[None, :]
                self._cut_static = S.cut_static(wl, prob, self.x[self.cut], h, fvals=fcut)
                self._jump_data = S.jump_data(wl, prob, self.x[nodes])
        b[self.uncut] = h * h * self._f_uncut
        if self.cut.size:
            nodes = self.cut[:, None] + self.node_offsets()[None, :]
            sides = self.side[nodes]
            J = S.jump_extension(wl, prob, None, grad_lo_cut, data=self._jump_data)
            terms = S.cut_terms(wl, prob, self.x[self.cut], h, sides, J, static=self._cut_static)
            self._cut_terms = terms
            b[self.cut] = -h * h * terms["K"]
        # Dirichlet neighbours
        g = np.zeros(self.N)
        bnd = ~self.interior
        g[bnd] = prob.g(self.x[bnd])
        self.gbnd = g
        ip = np.nonzero(self.interior)[0]
        for a in range(d):
            for sgn in (1, -1):
                q = ip + sgn * self.stride[a]
                isb = bnd[q]
                cf = self.cface[a][ip] if sgn == 1 else self.cface[a][q]
                b[ip[isb]] += cf[isb] * g[q[isb]]
        return b

    def kdiag(self):
        """Diagonal of the Helmholtz term, h^2 sum_s k^s v^s per interior node
        (uncut: h^2 k of its side; cut: with the cell's volume fractions), or
        None without one.  Needs the cut-cell data of rhs()."""
        wl = self.wl
        if wl.k_minus == 0.0 and wl.k_plus == 0.0:
            return None
        if not hasattr(self, "_kd"):
            h2 = self.h * self.h
            kd = np.zeros(self.N)
            kd[self.uncut] = h2 * np.where(self.side[self.uncut], wl.k_minus, wl.k_plus)
            if self.cut.size:
                st = self._cut_static
                kd[self.cut] = h2 * (st["km"] + st["kp"])
            self._kd = kd
        return self._kd

    def full_values(self, U):
        """Nodal values with the Dirichlet data filled in on the boundary."""
        out = U.copy()
        out[~self.interior] = self.gbnd[~self.interior]
        return out

    # ----------------------------------------------------------------- contrast
    def _extension_setup(self):
        """Everything of the low-side extension that depends only on the
        geometry (computed once, reused by every Picard iteration): the band
        |phi| < 6h of interior nodes two cells inside the box, the unit
        normals there (pointing away from the low side), the nodes whose q is
        known (low side) and the targets with their upwind neighbours."""
        if hasattr(self, "_ext"):
            return self._ext
        d, h, n = self.d, self.h, self.n
        lo = S.lo_side(self.wl)
        lo_mask = self.side if lo == 0 else ~self.side
        inner = self.interior.copy()
        for a in range(d):
            inner &= (self.idx[:, a] > 1) & (self.idx[:, a] < n - 1)
        cand = np.nonzero(inner)[0]
        band = np.abs(G.phi(self.wl, self.x[cand])) < 6.0 * h
        cand = cand[band]
        nrm = G.grad_phi(self.wl, self.x[cand])
        nn = np.sqrt((nrm * nrm).sum(axis=1, keepdims=True))
        nrm = nrm / np.where(nn > 0, nn, 1.0)
        if lo == 1:
            nrm = -nrm  # march from the low side outwards
        known = lo_mask[cand]
        ip, nrm_ip = cand[known], nrm[known]
        tgt, nrm_t = cand[~known], nrm[~known]
        # upwind neighbours: z - sign(n_a) e_a
        up_nb = np.stack([tgt - np.sign(nrm_t[:, a]).astype(np.int64) * self.stride[a]
                          for a in range(d)], axis=1)
        wts = np.abs(nrm_t)
        self._ext = {"lo_mask": lo_mask, "ip": ip, "nrm_ip": nrm_ip, "tgt": tgt, "up_nb": up_nb,
                     "wts": wts, "wsum": wts.sum(axis=1)}
        return self._ext

    def extend_lo(self, Ufull, sweeps=None):
        """Extend the low-mu side field across Gamma: constant normal
        derivative (upwind extrapolation of q = n.grad u), then linear
        extension of u with n.grad u = q.  Returns nodal array."""
        d, h = self.d, self.h
        ex = self._extension_setup()
        lo_mask, ip, nrm_ip = ex["lo_mask"], ex["ip"], ex["nrm_ip"]
        tgt, up_nb, wts, wsum = ex["tgt"], ex["up_nb"], ex["wts"], ex["wsum"]
        if sweeps is None:
            sweeps = 12
        # q = n . grad u on the low side (central differences if both
        # neighbours are on the low side, otherwise one-sided)
        q = np.zeros(self.N)
        for a in range(d):
            up, um = ip + self.stride[a], ip - self.stride[a]
            lu, lm = lo_mask[up], lo_mask[um]
            der = np.where(lu & lm, (Ufull[up] - Ufull[um]) / (2 * h),
                           np.where(lu, (Ufull[up] - Ufull[ip]) / h,
                                    np.where(lm, (Ufull[ip] - Ufull[um]) / h, 0.0)))
            q[ip] += nrm_ip[:, a] * der
        for _ in range(sweeps):
            q[tgt] = (wts * q[up_nb]).sum(axis=1) / wsum
        u = Ufull.copy()
        for _ in range(sweeps):
            u[tgt] = (h * q[tgt] + (wts * u[up_nb]).sum(axis=1)) / wsum
        return u

    def grad_at_cut_nodes(self, field):
        """Central differences of a nodal field at the cut-cell nodes
        (one-sided where a neighbour would leave the grid)."""
        nodes = self.cut[:, None] + self.node_offsets()[None, :]
        gr = np.zeros(nodes.shape + (self.d,))
        for a in range(self.d):
            ia = self.idx[nodes, a]
            up = np.where(ia < self.n, nodes + self.stride[a], nodes)
            dn = np.where(ia > 0, nodes - self.stride[a], nodes)
            span = (np.where(ia < self.n, 1, 0) + np.where(ia > 0, 1, 0)) * self.h
            gr[..., a] = (field[up] - field[dn]) / span
        return gr

    def solve(self, tol=1e-12, picard_tol=1e-10, max_picard=60, precond="mg", verbose=False,
              glo_fn=None, require_converged=True):
        """Solve the grid system.  With a contrast, the lagged low-mu gradients
        are found by the Picard iteration, unless glo_fn(y[..., d]) supplies
        them directly (used by the patch test with the exact low-side field).
        self.converged records whether the iteration met picard_tol within
        max_picard iterations; if it did not, PicardNotConverged is raised
        unless require_converged is False (an unconverged solution must never
        stand in for the judge)."""
        d, n = self.d, self.n
        contrast = S.lo_side(self.wl) >= 0
        ncut_nodes = (self.cut.size, 2 * d + 1, d)
        glo = np.zeros(ncut_nodes) if contrast else None
        if contrast and glo_fn is not None:
            nodes = self.cut[:, None] + self.node_offsets()[None, :]
            glo = glo_fn(self.x[nodes])
        b = self.rhs(glo)
        kd = self.kdiag()
        U, it, rr = pcg(d, n, self.cface, b, tol=tol, precond=precond, kdiag=kd)
        self.pcg_iters = [it]
        self.picard_iters = 0
        self.picard_dU = 0.0
        self.converged = True
        if contrast and glo_fn is None:
            self.converged = False
            # Anderson-accelerated fixed point on the lagged gradients
            hist_x, hist_f = [], []
            x = glo.ravel()
            for k in range(max_picard):
                Uf = self.full_values(U)
                ext = self.extend_lo(Uf)
                gnew = self.grad_at_cut_nodes(ext).ravel()
                f = gnew - x
                hist_x.append(x.copy())
                hist_f.append(f.copy())
                if len(hist_x) > 6:
                    hist_x.pop(0)
                    hist_f.pop(0)
                if len(hist_f) > 1:
                    dF = np.stack([hist_f[i + 1] - hist_f[i] for i in range(len(hist_f) - 1)], axis=1)
                    dX = np.stack([hist_x[i + 1] - hist_x[i] for i in range(len(hist_x) - 1)], axis=1)
                    gam, *_ = np.linalg.lstsq(dF, f, rcond=None)
                    x_next = x + f - (dX + dF) @ gam
                else:
                    x_next = x + f
                U_old = U
                x = x_next
                b = self.rhs(x.reshape(ncut_nodes))
                U, it, rr = pcg(d, n, self.cface, b, u0=U_old, tol=tol, precond=precond, kdiag=kd)
                self.pcg_iters.append(it)
                self.picard_iters = k + 1
                dU = np.abs(U - U_old).max()
                if verbose:
                    print(f"picard {k}: max|dU| = {dU:.3e}, pcg {it}")
                self.picard_dU = dU
                if dU <= picard_tol * max(1.0, np.abs(U).max()):
                    self.converged = True
                    break
        self.U = U
        self.relres = rr
        if require_converged and not self.converged:
            raise PicardNotConverged(
                f"Picard iteration: max|dU| = {self.picard_dU:.3e} after {self.picard_iters} "
                f"iterations (tolerance {picard_tol:.1e} relative)")
        return self.full_values(U)

    def row_residual(self, Ufull):
        """(A U - b) at interior nodes, divided by h^2 mubar (the collocation
        residual normalisation); with equal coefficients this must equal the
        collocation residual of the same node values."""
        Uz = Ufull.copy()
        Uz[~self.interior] = 0.0
        b = self.rhs(None if S.lo_side(self.wl) < 0 else np.zeros((self.cut.size, 2 * self.d + 1, self.d)))
        AU = apply_A(self.d, self.n, self.cface, Uz, kdiag=self.kdiag())
        mubar = np.zeros(self.N)
        ip = np.nonzero(self.interior)[0]
        for a in range(self.d):
            mubar[ip] += self.cface[a][ip] + self.cface[a][ip - self.stride[a]]
        mubar /= 2 * self.d
        out = np.zeros(self.N)
        out[ip] = (AU[ip] - b[ip]) / (self.h ** 2 * mubar[ip])
        return out


def cache_dir() -> Path:
    """Directory of cached grid solutions: $NBM_ORACLE_CACHE, else a folder in
    the system's temporary directory."""
    p = Path(os.environ.get("NBM_ORACLE_CACHE", str(Path(tempfile.gettempdir()) / "nbm_oracle_cache")))
    p.mkdir(parents=True, exist_ok=True)
    return p


def solve_cached(wl: I.Workload, n: int, verbose=False):
    """Grid solution (full nodal array) for workload wl at n intervals, cached
    on disk by a hash of the problem-defining fields."""
    key = repr((wl.dim, wl.interface, wl.radius, wl.star_amp, wl.mu_minus, wl.mu_plus, wl.problem,
                wl.alpha_const, wl.beta_const, wl.fourier_seed, wl.fourier_kmax, tuple(wl.plane_n),
                wl.plane_c, tuple(wl.lin_a), tuple(wl.lin_b), wl.k_minus, wl.k_plus, wl.mu_kind,
                wl.phi_n, wl.phi_shape, n, "v3"))
    hsh = hashlib.sha1(key.encode()).hexdigest()[:16]
    f = cache_dir() / f"grid_{hsh}.npy"
    if f.exists():
        return np.load(f, allow_pickle=False)
    gs = GridSystem(wl, n)
    U = gs.solve(verbose=verbose)
    np.save(f, U, allow_pickle=False)
    return U


def interp_grid(U, n, d, x):
    """Multilinear interpolation of a nodal grid array at points x[m, d]."""
    h = 2.0 / n
    t = (x + 1.0) / h
    i0 = np.clip(np.floor(t).astype(np.int64), 0, n - 1)
    fr = t - i0
    out = np.zeros(x.shape[0])
    for m in range(1 << d):
        w = np.ones(x.shape[0])
        flat = np.zeros(x.shape[0], dtype=np.int64)
        for a in range(d):
            bit = (m >> a) & 1
            w *= fr[:, a] if bit else (1.0 - fr[:, a])
            flat += (i0[:, a] + bit) * (n + 1) ** a
        out += w * U[flat]
    return out
