"""Problem data for the oracle (FP64, numpy).

Paper Sec. 2: k^+- u^+- - div(mu^+- grad u^+-) = f^+- in Omega^+-, with
[u] = alpha and [mu d_n u] = beta on Gamma, Dirichlet data on the cube.  All
workloads here have k^+- = 0 and piecewise-constant mu.  Manufactured
solutions: the sphere problem of Sec. 4.1 (u^- = e^z, u^+ = cos x sin y) with
constant mu^- = 1, mu^+ = 10, and a 2-D analogue with u^- = e^(x+y),
u^+ = sin(pi x) cos(pi y), mu = 1.  The Fourier workload has no closed-form
solution.  [q] = q^+ - q^-, n points from Omega^- to Omega^+.
"""
from __future__ import annotations

import numpy as np

import nbm_inputs as I
from . import geometry as G


class Problem:
    def __init__(self, wl: I.Workload):
        self.wl = wl
        self.mu = (wl.mu_minus, wl.mu_plus)
        if wl.problem == I.PROB_FOURIER:
            k, a, b = I.fourier_modes(wl)
            self.k = k.astype(np.float64)
            self.a = a
            self.b = b

    # exact solutions (manufactured problems only) ---------------------------
    def has_exact(self) -> bool:
        return self.wl.problem != I.PROB_FOURIER

    def u_side(self, s: int, x):
        """u^s(x) for s = 0 (minus) or 1 (plus), defined on the whole box."""
        p = self.wl.problem
        if p == I.PROB_MMS_2D:
            return np.exp(x[..., 0] + x[..., 1]) if s == 0 else \
                np.sin(np.pi * x[..., 0]) * np.cos(np.pi * x[..., 1])
        if p == I.PROB_MMS_SPHERE:
            return np.exp(x[..., 2]) if s == 0 else np.cos(x[..., 0]) * np.sin(x[..., 1])
        if p == I.PROB_LINEAR:
            c = np.array(self.wl.lin_a if s == 0 else self.wl.lin_b)
            d = x.shape[-1]
            return x @ c[:d] + c[3]
        raise ValueError("no closed-form solution for this problem")

    def grad_u_side(self, s: int, x):
        p = self.wl.problem
        g = np.zeros_like(x)
        if p == I.PROB_MMS_2D:
            if s == 0:
                e = np.exp(x[..., 0] + x[..., 1])
                g[..., 0] = e
                g[..., 1] = e
            else:
                g[..., 0] = np.pi * np.cos(np.pi * x[..., 0]) * np.cos(np.pi * x[..., 1])
                g[..., 1] = -np.pi * np.sin(np.pi * x[..., 0]) * np.sin(np.pi * x[..., 1])
            return g
        if p == I.PROB_MMS_SPHERE:
            if s == 0:
                g[..., 2] = np.exp(x[..., 2])
            else:
                g[..., 0] = -np.sin(x[..., 0]) * np.sin(x[..., 1])
                g[..., 1] = np.cos(x[..., 0]) * np.cos(x[..., 1])
            return g
        if p == I.PROB_LINEAR:
            c = np.array(self.wl.lin_a if s == 0 else self.wl.lin_b)
            g[...] = c[:x.shape[-1]]
            return g
        raise ValueError("no closed-form solution for this problem")

    def u_exact(self, x):
        m = G.side_minus(self.wl, x)
        return np.where(m, self.u_side(0, x), self.u_side(1, x))

    # forcing ------------------------------------------------------------------
    def f_side(self, s: int, x):
        """f^s = -mu^s Laplacian(u^s) (manufactured) or the Fourier series."""
        p = self.wl.problem
        mu = self.mu[s]
        if p == I.PROB_MMS_2D:
            if s == 0:
                return -mu * 2.0 * np.exp(x[..., 0] + x[..., 1])
            return mu * 2.0 * np.pi ** 2 * np.sin(np.pi * x[..., 0]) * np.cos(np.pi * x[..., 1])
        if p == I.PROB_MMS_SPHERE:
            if s == 0:
                return -mu * np.exp(x[..., 2])
            return mu * 2.0 * np.cos(x[..., 0]) * np.sin(x[..., 1])
        if p == I.PROB_LINEAR:
            return np.zeros(x.shape[:-1])
        # f(x) = sum_k a_k cos(pi k.x) + b_k sin(pi k.x), in chunks of points
        flat = x.reshape(-1, x.shape[-1])
        out = np.empty(flat.shape[0])
        for i in range(0, flat.shape[0], 8192):
            ph = np.pi * (flat[i:i + 8192] @ self.k.T)
            out[i:i + 8192] = np.cos(ph) @ self.a + np.sin(ph) @ self.b
        return out.reshape(x.shape[:-1])

    def f_grid(self, n: int):
        """Fourier forcing at every node of the grid with n intervals per
        axis (x_a = -1 + 2 i_a / n), flat index i0 + (n+1) i1 + (n+1)^2 i2.

        The same series as f_side, summed by axes: with c_k = a_k - i b_k,
        a_k cos(pi k.x) + b_k sin(pi k.x) = Re(c_k e^{i pi k.x}) and
        e^{i pi k.x} = prod_a e^{i pi k_a x_a}, so the sum over modes is three
        contractions of the dense coefficient array C[k0, k1, k2] (zero
        where k is not a mode) with the per-axis tables e^{i pi k_a x_a}."""
        if self.wl.problem != I.PROB_FOURIER or self.wl.dim != 3:
            raise ValueError("f_grid serves the 3-D Fourier forcing")
        km = int(np.abs(self.k).max())
        C = np.zeros((2 * km + 1,) * 3, dtype=np.complex128)
        ki = self.k.astype(np.int64) + km
        C[ki[:, 0], ki[:, 1], ki[:, 2]] = self.a - 1j * self.b
        x = -1.0 + (2.0 / n) * np.arange(n + 1)
        E = np.exp(1j * np.pi * np.outer(np.arange(-km, km + 1), x))   # [k, i]
        T = np.tensordot(C, E, axes=([0], [0]))        # [k1, k2, i0]
        T = np.tensordot(T, E, axes=([0], [0]))        # [k2, i0, i1]
        T = np.tensordot(T, E, axes=([0], [0]))        # [i0, i1, i2]
        return np.ascontiguousarray(T.real.transpose(2, 1, 0)).ravel()

    # jump data on Gamma (arguments are points on or projected to Gamma) -------
    def alpha(self, y, n):
        if self.wl.problem == I.PROB_FOURIER:
            return np.full(y.shape[:-1], self.wl.alpha_const)
        return self.u_side(1, y) - self.u_side(0, y)

    def beta(self, y, n):
        if self.wl.problem == I.PROB_FOURIER:
            return np.full(y.shape[:-1], self.wl.beta_const)
        gp = (self.grad_u_side(1, y) * n).sum(axis=-1)
        gm = (self.grad_u_side(0, y) * n).sum(axis=-1)
        return self.mu[1] * gp - self.mu[0] * gm

    # Dirichlet data ----------------------------------------------------------
    def g(self, x):
        if self.wl.problem == I.PROB_FOURIER:
            return np.zeros(x.shape[:-1])
        return self.u_exact(x)
