/* Preconditioned conjugate gradients for the grid judge (oracle, FP64).
 *
 * TEST INFRASTRUCTURE ONLY: part of the CPU oracle, never linked into the
 * product library.
 *
 * Operator on the nodes of a uniform grid with n intervals per axis (d = 2 or
 * 3), Dirichlet nodes on the boundary held at zero (their data is moved to the
 * right-hand side by the caller):
 *     (A u)_p = sum_a  c_a[p]     (u_p - u_{p+e_a})
 *                    + c_a[p-e_a] (u_p - u_{p-e_a})
 * c_a[p] is the coefficient of the face between node p and p + e_a
 * (sum over the two sides of mu^s times the face fraction), plus an optional
 * non-negative diagonal kd[p] u_p (the Helmholtz term k^s v^s h^2 of the
 * row).  A is symmetric positive definite.  The multigrid levels below the
 * finest carry the face part only (the preconditioner stays SPD).  Preconditioners: Jacobi, or one symmetric geometric
 * multigrid V-cycle (damped Jacobi smoothing, trilinear interpolation P,
 * restriction P^T, coarse faces = harmonic mean along / weighted arithmetic
 * mean across the fine faces, coarse operator scaled by 2^(d-2)).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int d, n;            /* dimension, intervals per axis */
  int64_t N;           /* (n+1)^d nodes */
  int64_t s[3];        /* strides */
  double* c[3];        /* face coefficients */
  const double* kd;    /* diagonal term (finest level only) or NULL */
  double* diag;
  double scale;        /* operator scale factor */
} level_t;

static int64_t npow(int n, int d) { int64_t r = 1; for (int i = 0; i < d; ++i) r *= (n + 1); return r; }

static void unravel(const level_t* L, int64_t idx, int* i) {
  for (int a = 0; a < L->d; ++a) { i[a] = (int)(idx % (L->n + 1)); idx /= (L->n + 1); }
}

static int interior(const level_t* L, const int* i) {
  for (int a = 0; a < L->d; ++a) if (i[a] <= 0 || i[a] >= L->n) return 0;
  return 1;
}

static void make_diag(level_t* L) {
  L->diag = (double*)calloc((size_t)L->N, sizeof(double));
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < L->N; ++p) {
    int i[3]; unravel(L, p, i);
    if (!interior(L, i)) continue;
    double dg = 0;
    for (int a = 0; a < L->d; ++a) dg += L->c[a][p] + L->c[a][p - L->s[a]];
    if (L->kd) dg += L->kd[p];
    L->diag[p] = dg * L->scale;
  }
}

static void apply(const level_t* L, const double* u, double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < L->N; ++p) {
    int i[3]; unravel(L, p, i);
    if (!interior(L, i)) { out[p] = 0.0; continue; }
    double acc = 0.0;
    for (int a = 0; a < L->d; ++a) {
      int64_t st = L->s[a];
      double up = (i[a] + 1 < L->n) ? u[p + st] : 0.0;
      double um = (i[a] - 1 > 0) ? u[p - st] : 0.0;
      acc += L->c[a][p] * (u[p] - up) + L->c[a][p - st] * (u[p] - um);
    }
    if (L->kd) acc += L->kd[p] * u[p];
    out[p] = acc * L->scale;
  }
}

static double dot(const double* a, const double* b, int64_t N) {
  double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
  for (int64_t p = 0; p < N; ++p) s += a[p] * b[p];
  return s;
}

/* coarse level from fine level */
static void coarsen(const level_t* F, level_t* C) {
  C->d = F->d; C->n = F->n / 2; C->N = npow(C->n, C->d);
  C->s[0] = 1; C->s[1] = C->n + 1; C->s[2] = (int64_t)(C->n + 1) * (C->n + 1);
  C->scale = F->scale * pow(2.0, C->d - 2);
  for (int a = 0; a < C->d; ++a) C->c[a] = (double*)calloc((size_t)C->N, sizeof(double));
  for (int a = C->d; a < 3; ++a) C->c[a] = NULL;
#pragma omp parallel for schedule(static)
  for (int64_t P = 0; P < C->N; ++P) {
    int I[3]; unravel(C, P, I);
    for (int a = 0; a < C->d; ++a) {
      if (I[a] >= C->n) continue;
      double acc = 0.0, wsum = 0.0;
      int lo[3], hi[3];
      for (int b = 0; b < C->d; ++b) { lo[b] = (b == a) ? 0 : -1; hi[b] = (b == a) ? 0 : 1; }
      int t[3];
      for (t[2] = (C->d > 2 ? lo[2] : 0); t[2] <= (C->d > 2 ? hi[2] : 0); ++t[2])
        for (t[1] = lo[1]; t[1] <= hi[1]; ++t[1])
          for (t[0] = lo[0]; t[0] <= hi[0]; ++t[0]) {
            int fi[3]; int ok = 1; double w = 1.0;
            for (int b = 0; b < C->d; ++b) {
              fi[b] = 2 * I[b] + t[b];
              if (fi[b] < 0 || fi[b] > F->n) ok = 0;
              if (b != a) w *= (t[b] == 0) ? 0.5 : 0.25;
            }
            if (!ok) continue;
            int64_t q = 0;
            for (int b = 0; b < C->d; ++b) q += fi[b] * F->s[b];
            double x = F->c[a][q], y = F->c[a][q + F->s[a]];
            double hm = (x + y > 0) ? 2.0 * x * y / (x + y) : 0.0;
            acc += w * hm; wsum += w;
          }
      C->c[a][P] = wsum > 0 ? acc / wsum : 0.0;
    }
  }
  make_diag(C);
}

static void jacobi(const level_t* L, const double* b, double* x, double* tmp, int sweeps, double w) {
  for (int it = 0; it < sweeps; ++it) {
    apply(L, x, tmp);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < L->N; ++p)
      if (L->diag[p] > 0) x[p] += w * (b[p] - tmp[p]) / L->diag[p];
  }
}

static void restrict_pt(const level_t* F, const level_t* C, const double* r, double* rc) {
#pragma omp parallel for schedule(static)
  for (int64_t P = 0; P < C->N; ++P) {
    int I[3]; unravel(C, P, I);
    if (!interior(C, I)) { rc[P] = 0.0; continue; }
    double acc = 0.0;
    int t[3];
    for (t[2] = (C->d > 2 ? -1 : 0); t[2] <= (C->d > 2 ? 1 : 0); ++t[2])
      for (t[1] = -1; t[1] <= 1; ++t[1])
        for (t[0] = -1; t[0] <= 1; ++t[0]) {
          double w = 1.0; int64_t q = 0;
          for (int b = 0; b < C->d; ++b) { w *= (t[b] == 0) ? 1.0 : 0.5; q += (2 * I[b] + t[b]) * F->s[b]; }
          acc += w * r[q];
        }
    rc[P] = acc;
  }
}

static void prolong_add(const level_t* F, const level_t* C, const double* ec, double* x) {
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < F->N; ++p) {
    int i[3]; unravel(F, p, i);
    if (!interior(F, i)) continue;
    int c0[3], c1[3];
    for (int b = 0; b < F->d; ++b) { c0[b] = i[b] / 2; c1[b] = (i[b] + 1) / 2; }
    double acc = 0.0;
    int ncomb = 1 << F->d;
    for (int m = 0; m < ncomb; ++m) {
      double w = 1.0; int64_t q = 0;
      for (int b = 0; b < F->d; ++b) {
        int use1 = (m >> b) & 1;
        if (c0[b] == c1[b]) { if (use1) { w = 0; break; } q += c0[b] * C->s[b]; }
        else { w *= 0.5; q += (use1 ? c1[b] : c0[b]) * C->s[b]; }
      }
      if (w != 0.0) acc += w * ec[q];
    }
    x[p] += acc;
  }
}

typedef struct { int nlev; level_t lev[16]; double* work[16][4]; } mg_t;

static void vcycle(mg_t* M, int k, const double* b, double* x) {
  level_t* L = &M->lev[k];
  double** w = M->work[k];
  memset(x, 0, sizeof(double) * (size_t)L->N);
  if (k == M->nlev - 1) { jacobi(L, b, x, w[0], 60, 0.8); return; }
  jacobi(L, b, x, w[0], 2, 0.8);
  apply(L, x, w[0]);
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < L->N; ++p) w[0][p] = b[p] - w[0][p];
  level_t* C = &M->lev[k + 1];
  restrict_pt(L, C, w[0], M->work[k + 1][2]);
  vcycle(M, k + 1, M->work[k + 1][2], M->work[k + 1][3]);
  prolong_add(L, C, M->work[k + 1][3], x);
  /* post-smoothing: continue the iteration from x */
  jacobi(L, b, x, w[0], 2, 0.8);
}

int nbm_oracle_pcg(int d, int n, const double* cface, const double* kdiag, const double* b, double* u,
                   double tol, int maxit, int precond, int* iters_out, double* relres_out) {
  if (d < 2 || d > 3 || n < 4) return -1;
  mg_t M; memset(&M, 0, sizeof(M));
  level_t* L0 = &M.lev[0];
  L0->d = d; L0->n = n; L0->N = npow(n, d); L0->scale = 1.0;
  L0->s[0] = 1; L0->s[1] = n + 1; L0->s[2] = (int64_t)(n + 1) * (n + 1);
  for (int a = 0; a < d; ++a) L0->c[a] = (double*)(cface + (int64_t)a * L0->N);
  L0->kd = kdiag;
  make_diag(L0);
  M.nlev = 1;
  if (precond == 1) {
    while (M.lev[M.nlev - 1].n > 4 && M.lev[M.nlev - 1].n % 2 == 0 && M.nlev < 16) {
      coarsen(&M.lev[M.nlev - 1], &M.lev[M.nlev]);
      M.nlev++;
    }
  }
  for (int k = 0; k < M.nlev; ++k)
    for (int j = 0; j < 4; ++j) M.work[k][j] = (double*)calloc((size_t)M.lev[k].N, sizeof(double));
  int64_t N = L0->N;
  double *r = (double*)calloc(N, 8), *z = (double*)calloc(N, 8), *pp = (double*)calloc(N, 8),
         *q = (double*)calloc(N, 8);
  /* zero the boundary entries of the guess */
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < N; ++p) { int i[3]; unravel(L0, p, i); if (!interior(L0, i)) u[p] = 0.0; }
  apply(L0, u, q);
  double bn = 0.0;
#pragma omp parallel for reduction(+ : bn) schedule(static)
  for (int64_t p = 0; p < N; ++p) {
    int i[3]; unravel(L0, p, i);
    double bb = interior(L0, i) ? b[p] : 0.0;
    r[p] = bb - q[p];
    bn += bb * bb;
  }
  bn = sqrt(bn);
  if (bn == 0.0) bn = 1.0;
  int it = 0;
  double rz = 0.0, res = sqrt(dot(r, r, N)) / bn;
  while (res > tol && it < maxit) {
    if (precond == 1) vcycle(&M, 0, r, z);
    else {
#pragma omp parallel for schedule(static)
      for (int64_t p = 0; p < N; ++p) z[p] = L0->diag[p] > 0 ? r[p] / L0->diag[p] : 0.0;
    }
    double rz_new = dot(r, z, N);
    if (it == 0) memcpy(pp, z, sizeof(double) * N);
    else {
      double beta = rz_new / rz;
#pragma omp parallel for schedule(static)
      for (int64_t p = 0; p < N; ++p) pp[p] = z[p] + beta * pp[p];
    }
    rz = rz_new;
    apply(L0, pp, q);
    double alpha = rz / dot(pp, q, N);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < N; ++p) { u[p] += alpha * pp[p]; r[p] -= alpha * q[p]; }
    res = sqrt(dot(r, r, N)) / bn;
    ++it;
  }
  *iters_out = it;
  *relres_out = res;
  free(r); free(z); free(pp); free(q);
  free(L0->diag);
  for (int k = 1; k < M.nlev; ++k) { for (int a = 0; a < d; ++a) free(M.lev[k].c[a]); free(M.lev[k].diag); }
  for (int k = 0; k < M.nlev; ++k) for (int j = 0; j < 4; ++j) free(M.work[k][j]);
  return 0;
}

/* y = A u (for tests of symmetry and of the assembled rows) */
int nbm_oracle_apply(int d, int n, const double* cface, const double* kdiag, const double* u, double* y) {
  level_t L; memset(&L, 0, sizeof(L));
  L.d = d; L.n = n; L.N = npow(n, d); L.scale = 1.0;
  L.s[0] = 1; L.s[1] = n + 1; L.s[2] = (int64_t)(n + 1) * (n + 1);
  for (int a = 0; a < d; ++a) L.c[a] = (double*)(cface + (int64_t)a * L.N);
  L.kd = kdiag;
  apply(&L, u, y);
  return 0;
}
