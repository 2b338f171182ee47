// Cut-cell geometry and residual assembly on the device (FP64).
// Cell C_p = x_p + [-h/2, h/2]^d; the level set is interpolated linearly on
// simplices (faces: segment / two triangles on the corner 0-3 diagonal;
// cells: two triangles / six Kuhn tetrahedra) and clipped in closed form.
#pragma once
#include "nbm_device.hpp"

namespace nbm {

// fraction of a segment / triangle / tetrahedron where the linear interpolant
// of the vertex values is negative (a zero value counts as non-negative)
__device__ inline double seg_neg(double a, double b) {
  bool na = a < 0.0, nb_ = b < 0.0;
  if (na && nb_) return 1.0;
  if (!na && !nb_) return 0.0;
  return na ? a / (a - b) : b / (b - a);
}

__device__ inline double tri_neg(double v0, double v1, double v2) {
  double v[3] = {v0, v1, v2};
  int k = (v0 < 0.0) + (v1 < 0.0) + (v2 < 0.0);
  if (k == 0) return 0.0;
  if (k == 3) return 1.0;
  // the vertex alone on its side
  int lone = 0;
  for (int i = 0; i < 3; ++i)
    if ((k == 1) == (v[i] < 0.0)) lone = i;
  double a = v[lone], b = v[(lone + 1) % 3], c = v[(lone + 2) % 3];
  double corner = a * a / ((a - b) * (a - c));
  return k == 1 ? corner : 1.0 - corner;
}

__device__ inline double tet_neg(const double* v) {
  int k = 0;
  for (int i = 0; i < 4; ++i) k += v[i] < 0.0;
  if (k == 0) return 0.0;
  if (k == 4) return 1.0;
  if (k == 1 || k == 3) {
    int lone = 0;
    for (int i = 0; i < 4; ++i)
      if ((k == 1) == (v[i] < 0.0)) lone = i;
    double a = v[lone], den = 1.0;
    for (int i = 0; i < 4; ++i)
      if (i != lone) den *= (a - v[i]);
    double corner = a * a * a / den;
    return k == 1 ? corner : 1.0 - corner;
  }
  double A = 0, B = 0, C = 0, E = 0;
  int ineg = 0, ipos = 0;
  for (int i = 0; i < 4; ++i) {
    if (v[i] < 0.0) { if (ineg++ == 0) A = -v[i]; else B = -v[i]; }
    else { if (ipos++ == 0) C = v[i]; else E = v[i]; }
  }
  double num = C * E * (A * A + A * B + B * B) + (C + E) * A * B * (A + B) + A * A * B * B;
  double den = (C + A) * (E + A) * (C + B) * (E + B);
  return num / den;
}

template <int D>
__device__ inline void crossing(const double* Pa, const double* Pb, double fa, double fb, double* q) {
  double t = fa / (fa - fb);
  for (int i = 0; i < D; ++i) q[i] = Pa[i] + t * (Pb[i] - Pa[i]);
}

__device__ inline double tri_area3(const double* a, const double* b, const double* c) {
  double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
  double w[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
  double cx = u[1] * w[2] - u[2] * w[1], cy = u[2] * w[0] - u[0] * w[2], cz = u[0] * w[1] - u[1] * w[0];
  return 0.5 * sqrt(cx * cx + cy * cy + cz * cz);
}

// zero set of a linear function in a triangle (2-D): accumulate length and
// length-weighted midpoint
__device__ inline void iface_tri(const double (*P)[3], const double* f, double& meas, double* mom) {
  int k = (f[0] < 0.0) + (f[1] < 0.0) + (f[2] < 0.0);
  if (k == 0 || k == 3) return;
  int lone = 0;
  for (int i = 0; i < 3; ++i)
    if ((k == 1) == (f[i] < 0.0)) lone = i;
  int j = (lone + 1) % 3, l = (lone + 2) % 3;
  double q1[3], q2[3];
  crossing<2>(P[lone], P[j], f[lone], f[j], q1);
  crossing<2>(P[lone], P[l], f[lone], f[l], q2);
  double len = sqrt((q1[0] - q2[0]) * (q1[0] - q2[0]) + (q1[1] - q2[1]) * (q1[1] - q2[1]));
  meas += len;
  mom[0] += len * 0.5 * (q1[0] + q2[0]);
  mom[1] += len * 0.5 * (q1[1] + q2[1]);
}

// zero polygon of a linear function in a tetrahedron: accumulate area and
// area-weighted centroid
__device__ inline void iface_tet(const double (*P)[3], const double* f, double& meas, double* mom) {
  int k = 0;
  for (int i = 0; i < 4; ++i) k += f[i] < 0.0;
  if (k == 0 || k == 4) return;
  if (k == 1 || k == 3) {
    int lone = 0;
    for (int i = 0; i < 4; ++i)
      if ((k == 1) == (f[i] < 0.0)) lone = i;
    double q[3][3];
    int t = 0;
    for (int i = 0; i < 4; ++i)
      if (i != lone) crossing<3>(P[lone], P[i], f[lone], f[i], q[t++]);
    double ar = tri_area3(q[0], q[1], q[2]);
    meas += ar;
    for (int a = 0; a < 3; ++a) mom[a] += ar * (q[0][a] + q[1][a] + q[2][a]) / 3.0;
    return;
  }
  int ng[2], ps[2], a_ = 0, b_ = 0;
  for (int i = 0; i < 4; ++i) {
    if (f[i] < 0.0) ng[a_++] = i; else ps[b_++] = i;
  }
  double qac[3], qae[3], qbe[3], qbc[3];
  crossing<3>(P[ng[0]], P[ps[0]], f[ng[0]], f[ps[0]], qac);
  crossing<3>(P[ng[0]], P[ps[1]], f[ng[0]], f[ps[1]], qae);
  crossing<3>(P[ng[1]], P[ps[1]], f[ng[1]], f[ps[1]], qbe);
  crossing<3>(P[ng[1]], P[ps[0]], f[ng[1]], f[ps[0]], qbc);
  double a1 = tri_area3(qac, qae, qbe), a2 = tri_area3(qac, qbe, qbc);
  meas += a1 + a2;
  for (int a = 0; a < 3; ++a)
    mom[a] += a1 * (qac[a] + qae[a] + qbe[a]) / 3.0 + a2 * (qac[a] + qbe[a] + qbc[a]) / 3.0;
}

struct CutGeom {
  double aneg[6];   // face fraction in Omega^-, face order +x0, -x0, +x1, ...
  double vneg;      // volume fraction in Omega^-
  double gamma;     // interface measure / h^(d-1)
  double cen[3];    // interface centroid
};

template <int D>
__device__ inline void cut_geometry(const Problem& P, const double* xc, double h, CutGeom& G) {
  constexpr int NC = 1 << D;
  double cp[NC][3], cf[NC];
  for (int c = 0; c < NC; ++c) {
    for (int a = 0; a < D; ++a) cp[c][a] = xc[a] + h * ((((c >> a) & 1) ? 0.5 : -0.5));
    for (int a = D; a < 3; ++a) cp[c][a] = 0.0;
    cf[c] = phi_at<D>(P, cp[c]);
  }
  for (int a = 0; a < D; ++a) {
    for (int sgn = 0; sgn < 2; ++sgn) {
      int ids[4];
      int nf = 1 << (D - 1);
      for (int m = 0; m < nf; ++m) {
        int c = sgn == 0 ? (1 << a) : 0;
        int t = 0;
        for (int b = 0; b < D; ++b) {
          if (b == a) continue;
          if ((m >> t) & 1) c |= 1 << b;
          ++t;
        }
        ids[m] = c;
      }
      double fr;
      if (D == 2) fr = seg_neg(cf[ids[0]], cf[ids[1]]);
      else fr = 0.5 * (tri_neg(cf[ids[0]], cf[ids[1]], cf[ids[3]]) + tri_neg(cf[ids[0]], cf[ids[2]], cf[ids[3]]));
      G.aneg[2 * a + sgn] = fr;
    }
  }
  double meas = 0.0, mom[3] = {0.0, 0.0, 0.0};
  if (D == 2) {
    const int tris[2][3] = {{0, 1, 3}, {0, 2, 3}};
    double v = 0.0;
    for (int t = 0; t < 2; ++t) {
      double Pt[3][3], ft[3];
      for (int i = 0; i < 3; ++i) {
        for (int a = 0; a < 3; ++a) Pt[i][a] = cp[tris[t][i]][a];
        ft[i] = cf[tris[t][i]];
      }
      v += tri_neg(ft[0], ft[1], ft[2]);
      iface_tri(Pt, ft, meas, mom);
    }
    G.vneg = 0.5 * v;
    G.gamma = meas / h;
  } else {
    const int tets[6][4] = {{0, 1, 3, 7}, {0, 1, 5, 7}, {0, 2, 3, 7}, {0, 2, 6, 7}, {0, 4, 5, 7}, {0, 4, 6, 7}};
    double v = 0.0;
    for (int t = 0; t < 6; ++t) {
      double Pt[4][3], ft[4];
      for (int i = 0; i < 4; ++i) {
        for (int a = 0; a < 3; ++a) Pt[i][a] = cp[tets[t][i]][a];
        ft[i] = cf[tets[t][i]];
      }
      v += tet_neg(ft);
      iface_tet(Pt, ft, meas, mom);
    }
    G.vneg = v / 6.0;
    G.gamma = meas / (h * h);
  }
  for (int a = 0; a < 3; ++a) G.cen[a] = meas > 0.0 ? mom[a] / meas : 0.0;
}

// Jump extension J(y) = alpha(pi y) + dist(y) j, j from beta and (with a
// coefficient contrast) the lagged low-mu normal derivative n . glo.
template <int D>
__device__ inline double jump_ext(const Problem& P, const double* y, const double* glo) {
  double pi[3], dist, n[3];
  project<D>(P, y, pi, dist, n);
  double al = alpha_at<D>(P, pi), be = beta_at<D>(P, pi, n);
  double mm = mu_at<double, D>(P, 0, pi), mp = mu_at<double, D>(P, 1, pi), j;
  if (P.lo < 0) {
    j = be / mm;
  } else {
    double gl = 0.0;
    for (int a = 0; a < D; ++a) gl += n[a] * glo[a];
    j = P.lo == 0 ? be / mp + (mm / mp - 1.0) * gl : be / mm + (1.0 - mp / mm) * gl;
  }
  return al + dist * j;
}

}  // namespace nbm
