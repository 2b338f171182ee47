"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This module holds data only: workload descriptions, parameter initialisation,
Fourier-mode tables and random test points.  It contains none of the method's
arithmetic (no geometry, no discretisation, no network evaluation), so both the
oracle and the HIP path may import it without sharing any computation.

Workloads follow the problem statement of the paper (Sec. 2: interface problem
with jumps [u]=alpha, [mu d_n u]=beta, Dirichlet box) and the numerical results
section (Sec. 4.1: sphere of radius 0.5 in [-1,1]^3, u^- = e^z, u^+ = cos x sin y,
two sine networks).  The five workloads are synthetic by construction.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

ACT_TANH = 0
ACT_SIN = 1
PREC_FP32 = 0
PREC_BF16 = 1
IFACE_SPHERE = 0   # circle in 2-D, sphere in 3-D, radius R
IFACE_STAR = 1     # |x| - 0.5 - amp * sin(5 theta) sin(4 psi)
IFACE_PLANE = 2    # n . x - c (test problems only)
IFACE_GRID = 3     # level set stored on a coarse mesh, interpolated (multi)linearly
PROB_MMS_2D = 0    # u^- = exp(x+y), u^+ = sin(pi x) cos(pi y)
PROB_MMS_SPHERE = 1  # u^- = exp(z), u^+ = cos(x) sin(y)
PROB_FOURIER = 2   # f^- = f^+ = seeded Fourier series, alpha, beta constants, g = 0
PROB_LINEAR = 3    # u^- = a.x + a0, u^+ = b.x + b0 (patch tests only)
MU_CONST = 0       # mu^-+ constants
MU_PAPER = 1       # mu^- = y^2 ln(x + 2) + 4, mu^+ = exp(-z) (Sec. 4.1)


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    dim: int
    width: int
    depth: int            # number of hidden layers of width `width`
    act: int
    prec: int
    h: float
    n_points: int         # interior collocation points per step
    n_boundary: int       # boundary collocation points per step
    interface: int
    radius: float
    star_amp: float
    mu_minus: float
    mu_plus: float
    problem: int
    alpha_const: float = 0.0
    beta_const: float = 0.0
    fourier_seed: int = 2
    fourier_kmax: float = 8.0
    steps: int = 200
    lr: float = 1e-3
    judge_n: int = 64     # intervals per axis of the grid judge
    plane_n: tuple = (0.6, 0.48, 0.64)   # IFACE_PLANE normal (unit)
    plane_c: float = 0.1                 # IFACE_PLANE offset
    lin_a: tuple = (0.3, -0.7, 0.2, 1.1)  # PROB_LINEAR u^- coefficients (x, y, z, const)
    lin_b: tuple = (-0.4, 0.9, 0.5, -0.6)  # PROB_LINEAR u^+ coefficients
    levels: int = 0       # implicit refinement levels: cells of side h, h/2, ..., h/2^levels
    k_minus: float = 0.0  # Helmholtz coefficients k^-+ of the term k u (>= 0)
    k_plus: float = 0.0
    mu_kind: int = 0      # 0: constant mu_minus / mu_plus; MU_PAPER: the variable coefficients of Sec. 4.1
    phi_n: int = 0        # IFACE_GRID: intervals per axis of the level-set mesh
    phi_shape: int = IFACE_STAR   # IFACE_GRID: the shape whose level set the mesh samples

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)

    @property
    def n_streams(self) -> int:
        return 2 * self.dim + 1

    @property
    def params_per_net(self) -> int:
        W, d, L = self.width, self.dim, self.depth
        return W * d + W + (L - 1) * (W * W + W) + W + 1

    @property
    def n_params(self) -> int:
        return 2 * self.params_per_net


def _nb(n, d, h):
    return int(round(n * d * h))


# 2-D plain NBM, FP32, circle, equal coefficients, tanh 16x2.
C1 = Workload("c1_circle2d_tanh16x2_fp32", 2, 16, 2, ACT_TANH, PREC_FP32, 1.0 / 32, 4096,
              _nb(4096, 2, 1.0 / 32), IFACE_SPHERE, 0.5, 0.0, 1.0, 1.0, PROB_MMS_2D,
              steps=200, judge_n=64)
# 3-D sphere, mu 1:10, tanh 64x3, FP32, fused backward.
C2 = Workload("c2_sphere3d_tanh64x3_fp32", 3, 64, 3, ACT_TANH, PREC_FP32, 1.0 / 128, 65536,
              _nb(65536, 3, 1.0 / 128), IFACE_SPHERE, 0.5, 0.0, 1.0, 10.0, PROB_MMS_SPHERE,
              steps=2000, judge_n=128)
# Same sphere problem, sin 128x4, BF16 GEMM operands.
C3 = Workload("c3_sphere3d_sin128x4_bf16", 3, 128, 4, ACT_SIN, PREC_BF16, 1.0 / 256, 262144,
              _nb(262144, 3, 1.0 / 256), IFACE_SPHERE, 0.5, 0.0, 1.0, 10.0, PROB_MMS_SPHERE,
              steps=2000, judge_n=256)
# Star interface, mu 1:100, Fourier forcing, sin 128x4 BF16, h = 1/1024.
C4 = Workload("c4_star3d_sin128x4_bf16", 3, 128, 4, ACT_SIN, PREC_BF16, 1.0 / 1024, 1048576,
              _nb(1048576, 3, 1.0 / 1024), IFACE_STAR, 0.5, 0.1, 1.0, 100.0, PROB_FOURIER,
              alpha_const=1.0, beta_const=0.0, steps=1000, judge_n=256)

# The paper's convergence workload (Sec. 4.1): sphere r = 0.5, u^- = e^z,
# u^+ = cos x sin y, mu^- = y^2 ln(x+2) + 4, mu^+ = e^-z, two sine networks of
# 5 hidden layers x 10 neurons (982 parameters); h = 2/N for N = 8..128.
PAPER = Workload("paper_sphere3d_varmu_sin10x5", 3, 10, 5, ACT_SIN, PREC_FP32, 1.0 / 32, 32768,
                 _nb(32768, 3, 1.0 / 32), IFACE_SPHERE, 0.5, 0.0, 4.0, 1.0, PROB_MMS_SPHERE,
                 steps=3000, judge_n=64, mu_kind=MU_PAPER)

WORKLOADS = {"c1": C1, "c2": C2, "c3": C3, "c4": C4, "paper": PAPER}


def xavier_params(wl: Workload, seed: int = 0, dtype=np.float64) -> np.ndarray:
    """Glorot-uniform weights, zero biases, packed net^- then net^+.

    Per net, in order: W1[W][d], b1[W], then for each hidden->hidden layer
    W_l[W][W], b_l[W], then w_out[W], b_out[1]; matrices row-major
    (row = output neuron).  One numpy PCG64 stream drives all draws.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    W, d, L = wl.width, wl.dim, wl.depth
    out = []
    for _net in range(2):
        shapes = [(W, d)] + [(W, W)] * (L - 1) + [(1, W)]
        for (fo, fi) in shapes:
            a = math.sqrt(6.0 / (fi + fo))
            out.append(rng.uniform(-a, a, size=fo * fi))
            out.append(np.zeros(fo))
    p = np.concatenate(out).astype(dtype)
    assert p.size == wl.n_params
    return p


def fourier_modes(wl: Workload):
    """Integer wave vectors k with 1 <= |k|_2 <= kmax, one of each +-k pair.

    The representative of a pair is the one whose first non-zero component is
    positive.  Enumeration order: k0, k1, k2 ascending from -kmax to kmax.
    Amplitudes a_k, b_k ~ N(0, 1/|k|^2) from a PCG64 stream seeded with
    `fourier_seed`.  Returns (k[int32, M x 3], a[float64 M], b[float64 M]).
    """
    km = int(math.floor(wl.fourier_kmax))
    ks = []
    for k0 in range(-km, km + 1):
        for k1 in range(-km, km + 1):
            for k2 in range(-km, km + 1):
                r2 = k0 * k0 + k1 * k1 + k2 * k2
                if r2 == 0 or r2 > wl.fourier_kmax ** 2:
                    continue
                first = k0 if k0 != 0 else (k1 if k1 != 0 else k2)
                if first > 0:
                    ks.append((k0, k1, k2))
    k = np.array(ks, dtype=np.int32)
    rng = np.random.Generator(np.random.PCG64(wl.fourier_seed))
    sd = 1.0 / np.sqrt((k.astype(np.float64) ** 2).sum(axis=1))
    a = rng.normal(size=len(k)) * sd
    b = rng.normal(size=len(k)) * sd
    return k, a, b


def phi_table(wl: Workload) -> np.ndarray:
    """Level-set values on the nodes -1 + 2 j / phi_n of a coarse mesh
    (IFACE_GRID workloads), axis 0 fastest: the level set of wl.phi_shape
    sampled at the nodes (star: |x| - R - amp sin(5 theta) sin(4 psi) with
    theta = atan2(y, x), psi = arccos(z/|x|), value -R at the origin; sphere:
    |x| - R; plane: n.x - c).  This is problem data, like a level set read
    from a file."""
    n, d = wl.phi_n, wl.dim
    ax = -1.0 + (2.0 / n) * np.arange(n + 1)
    g = np.meshgrid(*([ax] * d), indexing="ij")
    x = np.stack([m.transpose().ravel() for m in g], axis=-1)     # axis 0 fastest
    r = np.sqrt((x * x).sum(axis=1))
    if wl.phi_shape == IFACE_PLANE:
        return x @ np.array(wl.plane_n[:d]) - wl.plane_c
    if wl.phi_shape == IFACE_SPHERE:
        return r - wl.radius
    th = np.arctan2(x[:, 1], x[:, 0])
    cz = np.divide(x[:, 2], r, out=np.ones_like(r), where=r > 0)
    ps = np.arccos(np.clip(cz, -1.0, 1.0))
    v = r - wl.radius - wl.star_amp * np.sin(5.0 * th) * np.sin(4.0 * ps)
    return np.where(r > 0, v, -wl.radius)


LATTICE_BITS = 22


def lattice_points(n: int, d: int, lo: float, hi: float, seed: int) -> np.ndarray:
    """Uniform random points on the 2^-22 lattice inside [lo, hi]^d (float64).

    Every coordinate is an integer multiple of 2^-22, exact in float32 and
    float64; lo and hi must themselves be lattice values.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    q = float(2 ** LATTICE_BITS)
    jlo, jhi = int(round(lo * q)), int(round(hi * q))
    j = rng.integers(jlo, jhi + 1, size=(n, d))
    return j.astype(np.float64) / q


def boundary_lattice_points(n: int, d: int, seed: int) -> np.ndarray:
    """Uniform random points on the faces of [-1,1]^d, on the 2^-22 lattice."""
    rng = np.random.Generator(np.random.PCG64(seed))
    q = float(2 ** LATTICE_BITS)
    j = rng.integers(-(1 << LATTICE_BITS), (1 << LATTICE_BITS) + 1, size=(n, d))
    x = j.astype(np.float64) / q
    face = rng.integers(0, 2 * d, size=n)
    x[np.arange(n), face // 2] = np.where(face % 2 == 0, -1.0, 1.0)
    return x


def collocation_batch(wl: Workload, n: Optional[int] = None, nb: Optional[int] = None,
                      seed: int = 1):
    """Interior points in [-1+h, 1-h]^d and boundary points (float64 arrays)."""
    n = wl.n_points if n is None else n
    nb = wl.n_boundary if nb is None else nb
    pts = lattice_points(n, wl.dim, -1.0 + wl.h, 1.0 - wl.h, seed)
    bpts = boundary_lattice_points(nb, wl.dim, seed + 7919)
    return pts, bpts


def near_interface_points(wl: Workload, n: int, band: float, seed: int = 3) -> np.ndarray:
    """Lattice points whose radius lies within `band` of the sphere radius.

    Only meaningful for the sphere/circle interface; used to force cut cells
    into small test batches.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.normal(size=(n, wl.dim))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    r = wl.radius + rng.uniform(-band, band, size=(n, 1))
    x = v * r
    q = float(2 ** LATTICE_BITS)
    return np.round(x * q) / q
