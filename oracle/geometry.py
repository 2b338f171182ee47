"""Level-set geometry for the oracle (FP64, numpy).

Paper Sec. 2: a closed interface Gamma = {phi = 0} splits the cube into the
interior Omega^- (phi < 0) and exterior Omega^+ (phi >= 0, ties go to +).
Paper Sec. 3: the kernels need interface-cell crossings; here the level set is
interpolated linearly on simplices of each cell and clipped in closed form
(face fractions, volume fractions, interface measure and centroid).
"""
from __future__ import annotations

import itertools
import math

import numpy as np

import nbm_inputs as I


# ----------------------------------------------------------------------------
# level sets
# ----------------------------------------------------------------------------
_TABLES = {}


def _table(wl: I.Workload):
    key = (wl.phi_n, wl.phi_shape, wl.dim, wl.radius, wl.star_amp, tuple(wl.plane_n), wl.plane_c)
    if key not in _TABLES:
        _TABLES[key] = I.phi_table(wl)
    return _TABLES[key]


def phi_mesh(wl: I.Workload, x: np.ndarray) -> np.ndarray:
    """Level set stored on a coarse mesh (paper Sec. 3: a separate coarse mesh
    holds the level set that gives the kernels their geometry): multilinear
    interpolation of the nodal values on [-1, 1]^d with phi_n intervals per
    axis; points on the mesh's upper faces use the last cell."""
    n, d = wl.phi_n, x.shape[-1]
    tab = _table(wl)
    flat = x.reshape(-1, d)
    t = (flat + 1.0) * (n / 2.0)
    j = np.clip(np.floor(t).astype(np.int64), 0, n - 1)
    f = t - j
    out = np.zeros(flat.shape[0])
    for c in range(1 << d):
        w = np.ones(flat.shape[0])
        idx = np.zeros(flat.shape[0], dtype=np.int64)
        for a in range(d):
            bit = (c >> a) & 1
            w = w * (f[:, a] if bit else 1.0 - f[:, a])
            idx += (j[:, a] + bit) * (n + 1) ** a
        out += w * tab[idx]
    return out.reshape(x.shape[:-1])


def phi(wl: I.Workload, x: np.ndarray) -> np.ndarray:
    """Level set at points x[..., d] (FP64)."""
    if wl.interface == I.IFACE_GRID:
        return phi_mesh(wl, x)
    if wl.interface == I.IFACE_PLANE:
        nv = np.array(wl.plane_n[:x.shape[-1]])
        return x @ nv - wl.plane_c
    r = np.sqrt((x * x).sum(axis=-1))
    if wl.interface == I.IFACE_SPHERE:
        return r - wl.radius
    # star: |x| - 0.5 - amp sin(5 theta) sin(4 psi), theta = atan2(y, x),
    # psi = arccos(z/|x|); phi(0) = -0.5 by definition.
    theta = np.arctan2(x[..., 1], x[..., 0])
    with np.errstate(invalid="ignore", divide="ignore"):
        c = np.where(r > 0, x[..., 2] / np.where(r > 0, r, 1.0), 1.0)
    psi = np.arccos(np.clip(c, -1.0, 1.0))
    val = r - wl.radius - wl.star_amp * np.sin(5.0 * theta) * np.sin(4.0 * psi)
    return np.where(r > 0, val, -wl.radius)


def side_minus(wl: I.Workload, x: np.ndarray) -> np.ndarray:
    """True where a point belongs to Omega^- (phi < 0).

    For the circle/sphere the decision uses |x|^2 < R^2, which is exact for
    lattice points in FP64 (every square and their sum are exact)."""
    if wl.interface == I.IFACE_SPHERE:
        return (x * x).sum(axis=-1) < wl.radius * wl.radius
    return phi(wl, x) < 0.0


STAR_GRAD_STEP = 1e-6


def grad_phi(wl: I.Workload, x: np.ndarray) -> np.ndarray:
    """Gradient of phi: analytic for the sphere, central differences (step
    1e-6) for the star, whose angular factor is not smooth on the z-axis, and
    for the mesh level set, whose interpolant has kinks across mesh faces."""
    if wl.interface == I.IFACE_SPHERE:
        r = np.sqrt((x * x).sum(axis=-1, keepdims=True))
        return x / np.where(r > 0, r, 1.0)
    if wl.interface == I.IFACE_PLANE:
        return np.broadcast_to(np.array(wl.plane_n[:x.shape[-1]]), x.shape).copy()
    g = np.empty_like(x)
    for i in range(x.shape[-1]):
        e = np.zeros(x.shape[-1])
        e[i] = STAR_GRAD_STEP
        g[..., i] = (phi(wl, x + e) - phi(wl, x - e)) / (2 * STAR_GRAD_STEP)
    return g


def project(wl: I.Workload, y: np.ndarray):
    """One Newton step onto Gamma: pi(y) = y - phi grad(phi)/|grad(phi)|^2.

    Returns (pi(y), d(y) = phi/|grad phi|, unit normal at pi(y)).  Exact for
    the circle and the sphere."""
    p = phi(wl, y)
    g = grad_phi(wl, y)
    g2 = (g * g).sum(axis=-1)
    g2 = np.where(g2 > 0, g2, 1.0)
    pi = y - (p / g2)[..., None] * g
    dist = p / np.sqrt(g2)
    gn = grad_phi(wl, pi)
    nrm = np.sqrt((gn * gn).sum(axis=-1, keepdims=True))
    n = gn / np.where(nrm > 0, nrm, 1.0)
    return pi, dist, n


# ----------------------------------------------------------------------------
# closed-form clipping of a linear function on a simplex
# ----------------------------------------------------------------------------
def seg_neg_fraction(a, b):
    """Fraction of a segment where the linear interpolant of (a, b) is < 0."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    out = np.where((a < 0) & (b < 0), 1.0, 0.0)
    m1 = (a < 0) & (b >= 0)
    m2 = (b < 0) & (a >= 0)
    with np.errstate(invalid="ignore", divide="ignore"):
        out = np.where(m1, a / (a - b), out)
        out = np.where(m2, b / (b - a), out)
    return out


def _sorted_signs(vals):
    vals = np.asarray(vals, dtype=np.float64)
    return vals, (vals < 0).sum(axis=-1)


def tri_neg_fraction(v):
    """Area fraction of a triangle where the linear interpolant of the vertex
    values v[..., 3] is negative."""
    v, k = _sorted_signs(v)
    out = np.where(k == 3, 1.0, 0.0)
    neg = v < 0
    with np.errstate(invalid="ignore", divide="ignore"):
        # one negative vertex a: a^2 / ((a-b)(a-c))
        for i in range(3):
            j, l = [t for t in range(3) if t != i]
            a, b, c = v[..., i], v[..., j], v[..., l]
            one = (k == 1) & neg[..., i]
            out = np.where(one, a * a / ((a - b) * (a - c)), out)
            # two negative vertices, c = the non-negative one at index i
            two = (k == 2) & ~neg[..., i]
            out = np.where(two, 1.0 - a * a / ((a - b) * (a - c)), out)
    return out


def tet_neg_fraction(v):
    """Volume fraction of a tetrahedron where the linear interpolant of the
    vertex values v[..., 4] is negative (closed forms per sign pattern)."""
    v, k = _sorted_signs(v)
    out = np.where(k == 4, 1.0, 0.0)
    neg = v < 0
    with np.errstate(invalid="ignore", divide="ignore"):
        for i in range(4):
            o = [t for t in range(4) if t != i]
            a = v[..., i]
            b, c, e = v[..., o[0]], v[..., o[1]], v[..., o[2]]
            corner = a * a * a / ((a - b) * (a - c) * (a - e))
            out = np.where((k == 1) & neg[..., i], corner, out)
            out = np.where((k == 3) & ~neg[..., i], 1.0 - corner, out)
        for i, j in itertools.combinations(range(4), 2):
            o = [t for t in range(4) if t not in (i, j)]
            A, B = -v[..., i], -v[..., j]
            C, E = v[..., o[0]], v[..., o[1]]
            num = C * E * (A * A + A * B + B * B) + (C + E) * A * B * (A + B) + A * A * B * B
            den = (C + A) * (E + A) * (C + B) * (E + B)
            m = (k == 2) & neg[..., i] & neg[..., j]
            out = np.where(m, num / den, out)
    return out


def _cross_point(pa, pb, fa, fb):
    t = fa / (fa - fb)
    return pa + t[..., None] * (pb - pa)


def interface_in_triangle(P, f):
    """Zero segment of a linear function on a triangle.

    P[..., 3, 2] vertex coordinates, f[..., 3] values.  Returns (length,
    midpoint[..., 2]); zero length where there is no sign change (a vertex with
    f = 0 counts as non-negative)."""
    neg = f < 0
    k = neg.sum(axis=-1)
    length = np.zeros(f.shape[:-1])
    mid = np.zeros(f.shape[:-1] + (P.shape[-1],))
    with np.errstate(invalid="ignore", divide="ignore"):
        for i in range(3):
            j, l = [t for t in range(3) if t != i]
            # vertex i is alone on its side
            alone = ((k == 1) & neg[..., i]) | ((k == 2) & ~neg[..., i])
            p1 = _cross_point(P[..., i, :], P[..., j, :], f[..., i], f[..., j])
            p2 = _cross_point(P[..., i, :], P[..., l, :], f[..., i], f[..., l])
            seg = np.sqrt(((p1 - p2) ** 2).sum(axis=-1))
            length = np.where(alone, seg, length)
            mid = np.where(alone[..., None], 0.5 * (p1 + p2), mid)
    return np.nan_to_num(length), np.nan_to_num(mid)


def _tri_area3(a, b, c):
    return 0.5 * np.sqrt((np.cross(b - a, c - a) ** 2).sum(axis=-1))


def interface_in_tet(P, f):
    """Zero polygon of a linear function on a tetrahedron.

    P[..., 4, 3], f[..., 4].  Returns (area, centroid[..., 3])."""
    neg = f < 0
    k = neg.sum(axis=-1)
    area = np.zeros(f.shape[:-1])
    cen = np.zeros(f.shape[:-1] + (3,))
    with np.errstate(invalid="ignore", divide="ignore"):
        for i in range(4):
            o = [t for t in range(4) if t != i]
            alone = ((k == 1) & neg[..., i]) | ((k == 3) & ~neg[..., i])
            q = [_cross_point(P[..., i, :], P[..., t, :], f[..., i], f[..., t]) for t in o]
            ar = _tri_area3(q[0], q[1], q[2])
            area = np.where(alone, ar, area)
            cen = np.where(alone[..., None], (q[0] + q[1] + q[2]) / 3.0, cen)
        for i, j in itertools.combinations(range(4), 2):
            c, e = [t for t in range(4) if t not in (i, j)]
            two = (k == 2) & neg[..., i] & neg[..., j]
            qic = _cross_point(P[..., i, :], P[..., c, :], f[..., i], f[..., c])
            qie = _cross_point(P[..., i, :], P[..., e, :], f[..., i], f[..., e])
            qje = _cross_point(P[..., j, :], P[..., e, :], f[..., j], f[..., e])
            qjc = _cross_point(P[..., j, :], P[..., c, :], f[..., j], f[..., c])
            a1 = _tri_area3(qic, qie, qje)
            a2 = _tri_area3(qic, qje, qjc)
            c1 = (qic + qie + qje) / 3.0
            c2 = (qic + qje + qjc) / 3.0
            tot = a1 + a2
            cc = (a1[..., None] * c1 + a2[..., None] * c2) / np.where(tot > 0, tot, 1.0)[..., None]
            area = np.where(two, tot, area)
            cen = np.where(two[..., None], cc, cen)
    return np.nan_to_num(area), np.nan_to_num(cen)


# ----------------------------------------------------------------------------
# cell geometry
# ----------------------------------------------------------------------------
def corner_offsets(d: int) -> np.ndarray:
    """Corner offsets of the unit cell [-1/2, 1/2]^d; bit i of the corner index
    selects +1/2 along axis i."""
    return np.array([[((c >> i) & 1) - 0.5 for i in range(d)] for c in range(1 << d)])


def _kuhn_tets():
    """Six Kuhn simplices of the unit cube, as corner-index quadruples: walk
    from corner 0 to corner 7 adding one axis at a time."""
    tets = []
    for perm in itertools.permutations(range(3)):
        c = 0
        path = [c]
        for ax in perm:
            c |= 1 << ax
            path.append(c)
        tets.append(path)
    return tets


KUHN_TETS = _kuhn_tets()
# 2-D cell: two triangles sharing the diagonal corner 0 -> corner 3.
CELL_TRIS_2D = [[0, 1, 3], [0, 2, 3]]


def face_corner_ids(d: int, axis: int, plus: bool):
    """Corner indices of face F_{+-axis}, ordered by the remaining axes' bits
    (lowest remaining axis = fastest)."""
    others = [a for a in range(d) if a != axis]
    ids = []
    for m in range(1 << (d - 1)):
        c = (1 << axis) if plus else 0
        for t, a in enumerate(others):
            if (m >> t) & 1:
                c |= 1 << a
        ids.append(c)
    return ids


def cell_geometry(wl: I.Workload, xc: np.ndarray, h: float, phic: np.ndarray = None):
    """Cut-cell quantities of the cells x_p + [-h/2, h/2]^d.

    xc[n, d] cell centres.  Returns a dict with
      aneg[n, 2d]  fraction of face F (order +x0, -x0, +x1, -x1, ...) in Omega^-
      vneg[n]      volume fraction of the cell in Omega^-
      gamma[n]     |Gamma_h cap C_p| / h^(d-1)
      cen[n, d]    area-weighted centroid of Gamma_h cap C_p
    using the piecewise-linear interpolant of phi on simplices (faces: segment
    in 2-D, two triangles split on the corner-0 to corner-3 diagonal in 3-D;
    cells: two triangles in 2-D, six Kuhn tetrahedra in 3-D).
    """
    d = wl.dim
    n = xc.shape[0]
    off = corner_offsets(d)
    corners = xc[:, None, :] + h * off[None, :, :]
    if phic is None:
        phic = phi(wl, corners)
    aneg = np.zeros((n, 2 * d))
    for ax in range(d):
        for s, plus in enumerate((True, False)):
            ids = face_corner_ids(d, ax, plus)
            fv = phic[:, ids]
            if d == 2:
                fr = seg_neg_fraction(fv[:, 0], fv[:, 1])
            else:
                # face square corners (00, 10, 01, 11) -> triangles on 00-11
                fr = 0.5 * (tri_neg_fraction(fv[:, [0, 1, 3]]) + tri_neg_fraction(fv[:, [0, 2, 3]]))
            aneg[:, 2 * ax + s] = fr
    if d == 2:
        vneg = 0.5 * sum(tri_neg_fraction(phic[:, t]) for t in CELL_TRIS_2D)
        length = np.zeros(n)
        acc = np.zeros((n, 2))
        for t in CELL_TRIS_2D:
            L, m = interface_in_triangle(corners[:, t, :], phic[:, t])
            length += L
            acc += L[:, None] * m
        gamma = length / h
        cen = acc / np.where(length > 0, length, 1.0)[:, None]
    else:
        vneg = sum(tet_neg_fraction(phic[:, t]) for t in KUHN_TETS) / 6.0
        area = np.zeros(n)
        acc = np.zeros((n, 3))
        for t in KUHN_TETS:
            A, c = interface_in_tet(corners[:, t, :], phic[:, t])
            area += A
            acc += A[:, None] * c
        gamma = area / (h * h)
        cen = acc / np.where(area > 0, area, 1.0)[:, None]
    return {"aneg": aneg, "vneg": vneg, "gamma": gamma, "cen": cen, "phic": phic}
