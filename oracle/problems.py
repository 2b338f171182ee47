"""Problem data for the oracle (FP64, numpy).

Paper Sec. 2: k^+- u^+- - div(mu^+- grad u^+-) = f^+- in Omega^+-, with
[u] = alpha and [mu d_n u] = beta on Gamma, Dirichlet data on the cube.
mu piecewise constant, or the variable coefficients of Sec. 4.1
(mu^- = y^2 ln(x + 2) + 4, mu^+ = e^-z), and k >= 0 (k = 0: Poisson).  Manufactured
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
        self.k = (wl.k_minus, wl.k_plus)
        if wl.problem == I.PROB_FOURIER:
            k, a, b = I.fourier_modes(wl)
            self.kv = k.astype(np.float64)
            self.a = a
            self.b = b

    # diffusion coefficients --------------------------------------------------
    def mu_at(self, s: int, x):
        """mu^s(x): the constant, or the Sec. 4.1 functions."""
        if self.wl.mu_kind == I.MU_CONST:
            return np.full(x.shape[:-1], self.mu[s])
        if s == 0:
            return x[..., 1] ** 2 * np.log(x[..., 0] + 2.0) + 4.0
        return np.exp(-x[..., 2])

    def grad_mu(self, s: int, x):
        g = np.zeros_like(x)
        if self.wl.mu_kind == I.MU_CONST:
            return g
        if s == 0:
            g[..., 0] = x[..., 1] ** 2 / (x[..., 0] + 2.0)
            g[..., 1] = 2.0 * x[..., 1] * np.log(x[..., 0] + 2.0)
        else:
            g[..., 2] = -np.exp(-x[..., 2])
        return g

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
        """f^s = k^s u^s - div(mu^s grad u^s) = k^s u^s - mu^s Laplacian(u^s)
        - grad mu^s . grad u^s (manufactured) or the Fourier series."""
        p = self.wl.problem
        k = self.k[s]
        if self.wl.mu_kind != I.MU_CONST and p != I.PROB_FOURIER:
            f = self._f_const_mu(s, x, self.mu_at(s, x))
            return f - (self.grad_mu(s, x) * self.grad_u_side(s, x)).sum(axis=-1)
        return self._f_const_mu(s, x, self.mu[s])

    def _f_const_mu(self, s: int, x, mu):
        p = self.wl.problem
        k = self.k[s]
        if p == I.PROB_MMS_2D:
            if s == 0:
                lap = 2.0 * np.exp(x[..., 0] + x[..., 1])
            else:
                lap = -2.0 * np.pi ** 2 * np.sin(np.pi * x[..., 0]) * np.cos(np.pi * x[..., 1])
            return -mu * lap + (k * self.u_side(s, x) if k else 0.0)
        if p == I.PROB_MMS_SPHERE:
            lap = np.exp(x[..., 2]) if s == 0 else -2.0 * np.cos(x[..., 0]) * np.sin(x[..., 1])
            return -mu * lap + (k * self.u_side(s, x) if k else 0.0)
        if p == I.PROB_LINEAR:
            return k * self.u_side(s, x) if k else np.zeros(x.shape[:-1])
        # f(x) = sum_k a_k cos(pi k.x) + b_k sin(pi k.x), in chunks of points
        flat = x.reshape(-1, x.shape[-1])
        out = np.empty(flat.shape[0])
        for i in range(0, flat.shape[0], 8192):
            ph = np.pi * (flat[i:i + 8192] @ self.kv.T)
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
        km = int(np.abs(self.kv).max())
        C = np.zeros((2 * km + 1,) * 3, dtype=np.complex128)
        ki = self.kv.astype(np.int64) + km
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
        return self.mu_at(1, y) * gp - self.mu_at(0, y) * gm

    # Dirichlet data ----------------------------------------------------------
    def g(self, x):
        if self.wl.problem == I.PROB_FOURIER:
            return np.zeros(x.shape[:-1])
        return self.u_exact(x)
