"""Pins of the oracle geometry: closed-form simplex clipping checked against an
independent divided-difference formula, planar cells, and sphere/circle
volume and area sums against their closed forms (O(h^2) decay)."""
import math

import numpy as np
import pytest

import nbm_inputs as I
from oracle import geometry as G


def spline_fraction(v):
    """Fraction of a simplex where a linear function with distinct vertex
    values v is negative: the uniform measure of {phi < 0} is a B-spline in
    the values, F = sum_{i: v_i<0} (-v_i)^d / prod_{j != i} (v_j - v_i)."""
    d = len(v) - 1
    tot = 0.0
    for i, vi in enumerate(v):
        if vi < 0:
            den = 1.0
            for j, vj in enumerate(v):
                if j != i:
                    den *= (vj - vi)
            tot += (-vi) ** d / den
    return tot


@pytest.mark.parametrize("k", [3, 4])
def test_simplex_fraction_matches_spline_formula(k):
    rng = np.random.default_rng(11)
    V = rng.normal(size=(4000, k))
    f = G.tri_neg_fraction(V) if k == 3 else G.tet_neg_fraction(V)
    ref = np.array([spline_fraction(v) for v in V])
    assert np.max(np.abs(f - ref)) < 1e-9


def test_simplex_fraction_edge_cases():
    assert G.tri_neg_fraction(np.array([-1.0, 0.0, 0.0])) == pytest.approx(1.0)
    assert G.tri_neg_fraction(np.array([0.0, 0.0, 0.0])) == 0.0
    assert G.tri_neg_fraction(np.array([-1.0, 1.0, 0.0])) == pytest.approx(0.5)
    assert G.tet_neg_fraction(np.array([-1.0, -1.0, 0.0, 0.0])) == pytest.approx(1.0)
    assert G.tet_neg_fraction(np.array([-1.0, -1.0, 1.0, 1.0])) == pytest.approx(0.5)
    assert G.seg_neg_fraction(-1.0, 3.0) == pytest.approx(0.25)


def test_fraction_monte_carlo_tet():
    """Brute force: sample the tetrahedron uniformly."""
    rng = np.random.default_rng(5)
    v = np.array([-0.7, 0.2, -0.1, 0.9])
    lam = rng.dirichlet(np.ones(4), size=400000)
    mc = np.mean(lam @ v < 0)
    assert abs(G.tet_neg_fraction(v) - mc) < 3e-3


def test_planar_cell_exact():
    wl = I.C2.replace(interface=I.IFACE_PLANE, plane_n=(1.0, 0.0, 0.0), plane_c=0.013)
    h = 0.05
    xc = np.array([[0.0, 0.2, -0.3]])
    g = G.cell_geometry(wl, xc, h)
    frac = (0.013 - (-h / 2)) / h
    assert g["vneg"][0] == pytest.approx(frac, abs=1e-14)
    assert g["gamma"][0] == pytest.approx(1.0, abs=1e-12)
    assert g["cen"][0, 0] == pytest.approx(0.013, abs=1e-14)
    # face +x entirely in Omega^+, face -x entirely in Omega^-, side faces cut
    assert g["aneg"][0, 0] == 0.0 and g["aneg"][0, 1] == 1.0
    assert g["aneg"][0, 2] == pytest.approx(frac, abs=1e-14)


def test_oblique_plane_area_and_volume():
    """Oblique plane through a cube: the cross-section area and the volume
    below follow from the exact integrals of the linear function."""
    n = np.array([0.6, 0.48, 0.64])
    wl = I.C2.replace(interface=I.IFACE_PLANE, plane_n=tuple(n), plane_c=0.0)
    h = 1.0
    g = G.cell_geometry(wl, np.zeros((1, 3)), h)
    # plane through the centre: half the volume, by symmetry
    assert g["vneg"][0] == pytest.approx(0.5, abs=1e-13)
    # Monte Carlo area check via the coarea formula on a thin slab
    rng = np.random.default_rng(1)
    X = rng.uniform(-0.5, 0.5, size=(2_000_000, 3))
    eps = 0.01
    area_mc = np.mean(np.abs(X @ n) < eps / 2) / eps
    assert g["gamma"][0] == pytest.approx(area_mc, rel=0.02)


@pytest.mark.parametrize("dim", [2, 3])
def test_sphere_volume_and_area_converge(dim):
    wl = (I.C1 if dim == 2 else I.C2)
    errs_v, errs_a = [], []
    for n in (16, 32):
        h = 2.0 / n
        ax = -1 + h / 2 + h * np.arange(n)
        X = np.stack(np.meshgrid(*([ax] * dim), indexing="ij"), -1).reshape(-1, dim)
        g = G.cell_geometry(wl, X, h)
        R = wl.radius
        vol = g["vneg"].sum() * h ** dim
        area = g["gamma"].sum() * h ** (dim - 1)
        if dim == 2:
            errs_v.append(abs(vol - math.pi * R * R))
            errs_a.append(abs(area - 2 * math.pi * R))
        else:
            errs_v.append(abs(vol - 4.0 / 3.0 * math.pi * R ** 3))
            errs_a.append(abs(area - 4 * math.pi * R * R))
    assert errs_v[1] < errs_v[0] / 3.0 and errs_v[1] < 5e-3
    assert errs_a[1] < errs_a[0] / 3.0 and errs_a[1] < 2e-2


def test_projection_exact_on_sphere():
    wl = I.C2
    rng = np.random.default_rng(3)
    y = rng.uniform(-1, 1, size=(100, 3))
    pi, dist, n = G.project(wl, y)
    assert np.allclose(np.linalg.norm(pi, axis=1), wl.radius, atol=1e-14)
    assert np.allclose(dist, np.linalg.norm(y, axis=1) - wl.radius, atol=1e-14)


def test_star_level_set_definition():
    """phi(0) = -0.5, and along the z-axis and the equator the angular factor
    vanishes (sin(4 psi) = 0 at psi = 0, pi/2)."""
    wl = I.C4
    assert G.phi(wl, np.zeros((1, 3)))[0] == -0.5
    p = np.array([[0.0, 0.0, 0.7], [0.3, 0.4, 0.0]])
    assert np.allclose(G.phi(wl, p), np.linalg.norm(p, axis=1) - 0.5, atol=1e-15)
    # at theta = pi/10, psi = pi/8: sin(5 theta) = 1, sin(4 psi) = 1
    th, ps, r = math.pi / 10, math.pi / 8, 0.55
    q = np.array([[r * math.sin(ps) * math.cos(th), r * math.sin(ps) * math.sin(th), r * math.cos(ps)]])
    assert G.phi(wl, q)[0] == pytest.approx(r - 0.5 - 0.1, abs=1e-14)


def _mesh_wl(shape, n, **kw):
    return I.C2.replace(interface=I.IFACE_GRID, phi_shape=shape, phi_n=n, **kw)


def test_mesh_level_set_interpolates_its_nodes():
    """The coarse-mesh level set equals its nodal values at the nodes, is
    linear along mesh edges and multilinear inside a cell (midpoint of a cell
    = mean of its 8 corners)."""
    wl = _mesh_wl(I.IFACE_STAR, 8)
    tab = I.phi_table(wl)
    n = 8
    rng = np.random.default_rng(4)
    j = rng.integers(0, n + 1, size=(50, 3))
    x = -1.0 + 2.0 * j / n
    flat = j[:, 0] + (n + 1) * j[:, 1] + (n + 1) ** 2 * j[:, 2]
    assert np.allclose(G.phi(wl, x), tab[flat], rtol=0, atol=1e-14)
    j = rng.integers(0, n, size=(50, 3))
    mid = -1.0 + 2.0 * (j + 0.5) / n
    corners = sum(tab[(j[:, 0] + a) + (n + 1) * (j[:, 1] + b) + (n + 1) ** 2 * (j[:, 2] + c)]
                  for a in (0, 1) for b in (0, 1) for c in (0, 1)) / 8.0
    assert np.allclose(G.phi(wl, mid), corners, rtol=0, atol=1e-14)
    t = rng.uniform(0, 1, size=50)
    e0 = -1.0 + 2.0 * j / n
    e1 = e0.copy()
    e1[:, 1] += 2.0 / n
    pe = G.phi(wl, (1 - t)[:, None] * e0 + t[:, None] * e1)
    assert np.allclose(pe, (1 - t) * G.phi(wl, e0) + t * G.phi(wl, e1), rtol=0, atol=1e-13)


def test_mesh_level_set_of_a_plane_is_the_plane():
    """Multilinear interpolation reproduces a linear function exactly, so a
    mesh sampling the plane gives the analytic plane's sides, cut-cell
    geometry and interface data."""
    wp = I.C2.replace(interface=I.IFACE_PLANE, plane_n=(0.6, 0.48, 0.64), plane_c=0.07)
    wm = _mesh_wl(I.IFACE_PLANE, 8, plane_n=(0.6, 0.48, 0.64), plane_c=0.07)
    x = I.lattice_points(4000, 3, -0.99, 0.99, seed=3)
    assert np.allclose(G.phi(wm, x), G.phi(wp, x), rtol=0, atol=1e-13)
    xc = x[np.abs(G.phi(wp, x)) < 0.02][:300]
    gp, gm = G.cell_geometry(wp, xc, 1 / 64), G.cell_geometry(wm, xc, 1 / 64)
    for k in ("aneg", "vneg", "gamma", "cen"):
        assert np.allclose(gp[k], gm[k], rtol=0, atol=1e-11), k


@pytest.mark.parametrize("dim", [2, 3])
def test_mesh_sphere_volume_converges(dim):
    """A mesh sampling the sphere (circle): the volume of Omega^- from the
    cells' simplex clipping approaches the closed form at second order as the
    level-set mesh is refined."""
    base = I.C1 if dim == 2 else I.C2
    h = 1.0 / 32
    xs = -1.0 + h * (np.arange(int(2 / h)) + 0.5)
    xc = np.stack(np.meshgrid(*([xs] * dim), indexing="ij"), axis=-1).reshape(-1, dim)
    exact = math.pi * 0.25 if dim == 2 else 4.0 / 3.0 * math.pi * 0.125
    errs = []
    for n in (8, 16, 32):
        wl = base.replace(interface=I.IFACE_GRID, phi_shape=I.IFACE_SPHERE, phi_n=n)
        near = np.abs(np.sqrt((xc * xc).sum(axis=1)) - 0.5) < 3 * h
        inside = (np.sqrt((xc * xc).sum(axis=1)) < 0.5) & ~near
        vol = (inside.sum() + G.cell_geometry(wl, xc[near], h)["vneg"].sum()) * h ** dim
        errs.append(abs(vol - exact))
    assert errs[1] < errs[0] / 3 and errs[2] < errs[1] / 2.5, errs
