/*
 * pair_oracle.c -- plain FP64 force-matched pair draft.
 *
 * TEST INFRASTRUCTURE ONLY (see lsd_oracle.c).  The paper's drafts are
 * lighter interatomic potentials than the target, fitted to reproduce its
 * forces; LSD accepts any draft force field, conservative or not (Sec. 3,
 * Sec. 4).  The fallback draft defined here is a central pair force whose
 * radial profile per unordered species pair is linear in its weights, so
 * force matching is a linear least-squares problem:
 *
 *   F_i    = - sum_(j, n) f_t(r) d / r,    d = q_j + n L - q_i,  r = |d| < rc
 *   f_t(r) = f_c(r) sum_{b=1..B} w_{t,b} sin(b pi r / rc) / r
 *   f_c(r) = (cos(pi r / rc) + 1) / 2
 *   t      = index of the unordered species pair {s_i, s_j}: for a <= b,
 *            t(a, b) = a S - a (a - 1) / 2 + (b - a)   (S species, S(S+1)/2
 *            types in the order (0,0), (0,1), .., (0,S-1), (1,1), ..)
 *
 * A positive f pushes i away from j.  F is linear in w: F_i = A_i w with
 *   A_i[d][t B + b-1] = - sum_(j, n) [t(s_i, s_j) = t] f_c(r) sin(b pi r/rc)/r * d_d / r,
 * and the weights minimise sum over frames and atoms |F_target - A w|^2.
 * ora_pair_forces evaluates the force sum directly; ora_pair_design builds
 * A; the two are separate loops.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

long ora_pairs_brute(int n, const double *x, double L, double rc, int32_t *out, long cap);
long ora_pairs_cells(int n, const double *x, double L, double rc, int32_t *out, long cap);

int ora_pair_types(int S) { return S * (S + 1) / 2; }

int ora_pair_type(int a, int b, int S) {
  if (a > b) { int t = a; a = b; b = t; }
  return a * S - a * (a - 1) / 2 + (b - a);
}

/* every ordered (i, j, image) within rc, as (i, j, nx, ny, nz) records */
static long pair_records(int n, const double *x, double L, double rc, int32_t **out) {
  int cells = floor(L / rc) >= 3;
  long np = cells ? ora_pairs_cells(n, x, L, rc, NULL, 0) : ora_pairs_brute(n, x, L, rc, NULL, 0);
  *out = (int32_t *)malloc(sizeof(int32_t) * 5 * (size_t)(np > 0 ? np : 1));
  if (cells) ora_pairs_cells(n, x, L, rc, *out, np);
  else ora_pairs_brute(n, x, L, rc, *out, np);
  return np;
}

static void separation(const double *x, double L, const int32_t *rec, double d[3], double *r) {
  int i = rec[0], j = rec[1];
  for (int a = 0; a < 3; ++a) d[a] = (x[3 * j + a] - x[3 * i + a]) + (double)rec[2 + a] * L;
  *r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
}

/* radial profile f_t(r) for one type's weights w[B] */
static double profile(const double *w, int B, double r, double rc) {
  const double pi = 3.14159265358979323846;
  double fc = 0.5 * (cos(pi * r / rc) + 1.0), s = 0.0;
  for (int b = 1; b <= B; ++b) s += w[b - 1] * sin(b * pi * r / rc) / r;
  return fc * s;
}

/* F[n][3] of the pair draft with weights w[T][B] */
void ora_pair_forces(int n, const double *x, double L, const int32_t *sp, int S, int B, double rc,
                     const double *w, double *F) {
  int32_t *rec;
  long np = pair_records(n, x, L, rc, &rec);
  memset(F, 0, sizeof(double) * 3 * (size_t)n);
  for (long p = 0; p < np; ++p) {
    const int32_t *q = &rec[5 * p];
    double d[3], r;
    separation(x, L, q, d, &r);
    int t = ora_pair_type(sp[q[0]], sp[q[1]], S);
    double f = profile(&w[(size_t)t * B], B, r, rc);
    for (int a = 0; a < 3; ++a) F[3 * q[0] + a] -= f * d[a] / r;
  }
  free(rec);
}

/* design matrix A[3n][T B] (row 3 i + d) of the forces in the weights */
void ora_pair_design(int n, const double *x, double L, const int32_t *sp, int S, int B, double rc,
                     double *A) {
  const double pi = 3.14159265358979323846;
  int P = ora_pair_types(S) * B;
  int32_t *rec;
  long np = pair_records(n, x, L, rc, &rec);
  memset(A, 0, sizeof(double) * 3 * (size_t)n * P);
  for (long p = 0; p < np; ++p) {
    const int32_t *q = &rec[5 * p];
    double d[3], r;
    separation(x, L, q, d, &r);
    int t = ora_pair_type(sp[q[0]], sp[q[1]], S);
    double fc = 0.5 * (cos(pi * r / rc) + 1.0);
    for (int b = 1; b <= B; ++b) {
      double g = fc * sin(b * pi * r / rc) / r;
      for (int a = 0; a < 3; ++a)
        A[(size_t)(3 * q[0] + a) * P + (size_t)t * B + (b - 1)] -= g * d[a] / r;
    }
  }
  free(rec);
}

/* The pair draft as a force field of the integrator and window code
 * (lsd_oracle.c, kind ORA_POT_EXT); its energy is never needed (0). */
typedef struct {
  int S, B;
  double rc;
  const double *w;
  const int32_t *species;
} ora_pair_ctx;

double ora_pair_ext(const void *ctx, int n, const double *x, double L, double *F) {
  const ora_pair_ctx *c = (const ora_pair_ctx *)ctx;
  ora_pair_forces(n, x, L, c->species, c->S, c->B, c->rc, c->w, F);
  return 0.0;
}
