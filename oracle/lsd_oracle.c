/*
 * lsd_oracle.c -- plain FP64 CPU oracle for Langevin Speculative Dynamics.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU product path may call, link
 * or load this file; only tests/, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header or constant table with the HIP
 * library: everything here is written out from the paper
 * ("Speculative Sampling For Faster Molecular Dynamics", arXiv 2606.02455)
 * and from the published definition of Philox4x32-10.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (see oracle/build.py).
 * -ffp-contract=off keeps every multiply and add separately rounded, so the
 * neighbour predicate below is the exact IEEE-754 binary64 expression.
 *
 * Conventions
 *   positions / momenta / forces: AoS double [n][3], atom-major.
 *   Cubic periodic box of edge L; positions are wrapped into [0, L) after
 *   every position update (A step), with integer image counters.
 *   "fu" (force unit) converts force*time into momentum and energy into
 *   mass*length^2/time^2 (1 in Lennard-Jones reduced units).
 *
 * Parity: every function is pinned by tests/test_oracle_*.py (finite
 * differences, closed forms, brute force, published test vectors, exact
 * stationary laws).  The message-passing potential lives in mpnn_oracle.c.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,        */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11): ten rounds of two  */
/* 32x32->64 multiplies with a Weyl-sequence key schedule.                   */
/* ------------------------------------------------------------------------ */
static const uint32_t PHILOX_MUL0 = 0xD2511F53u;
static const uint32_t PHILOX_MUL1 = 0xCD9E8D57u;
static const uint32_t PHILOX_WEYL0 = 0x9E3779B9u; /* golden ratio */
static const uint32_t PHILOX_WEYL1 = 0xBB67AE85u; /* sqrt(3) - 1 */

void ora_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                       uint32_t out[4]) {
  uint32_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += PHILOX_WEYL0;
      k1 += PHILOX_WEYL1;
    }
    uint64_t prod0 = (uint64_t)PHILOX_MUL0 * (uint64_t)x0;
    uint64_t prod1 = (uint64_t)PHILOX_MUL1 * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
    uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Random stream of the method (the paper only asks for xi ~ N(0, I), Eq.
 * aboba, and u ~ Uniform[0,1], Eq. reflectionVerify).  Reading fixed for this
 * implementation: the stream is keyed by the simulation step n being
 * produced, so a redraft after a rollback reuses the keys of flushed steps.
 *   key     = (seed low 32 bits, seed high 32 bits)
 *   counter = (local atom index or 0, n low, n high,
 *              replica << 8 | tag << 4 | block)
 *   tag 1 = Gaussian noise xi, tag 2 = acceptance uniform u.
 * Uniform from two words w_lo, w_hi: ((w_hi:w_lo >> 11) + 1) * 2^-53, in
 * (0, 1].  Normals by Box-Muller on the uniforms (w0,w1) and (w2,w3). */
#define ORA_TAG_XI 1u
#define ORA_TAG_U 2u

static double u53(uint32_t lo, uint32_t hi) {
  uint64_t x = ((uint64_t)hi << 32) | (uint64_t)lo;
  return (double)((x >> 11) + 1u) * (1.0 / 9007199254740992.0);
}

static void stream_words(uint64_t seed, uint32_t replica, uint64_t step,
                         uint32_t index, uint32_t tag, uint32_t block,
                         uint32_t w[4]) {
  uint32_t ctr[4] = {index, (uint32_t)step, (uint32_t)(step >> 32),
                     (replica << 8) | (tag << 4) | block};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  ora_philox4x32_10(ctr, key, w);
}

double ora_uniform(uint64_t seed, uint32_t replica, uint64_t step) {
  uint32_t w[4];
  stream_words(seed, replica, step, 0u, ORA_TAG_U, 0u, w);
  return u53(w[0], w[1]);
}

/* xi[n][3] for step `step` of replica `replica`; component (i, d) takes
 * Box-Muller output d&1 of block d>>1 at counter index i. */
void ora_normals(uint64_t seed, uint32_t replica, uint64_t step, int n,
                 double *xi) {
  const double two_pi = 6.283185307179586476925286766559;
  for (int i = 0; i < n; ++i) {
    for (uint32_t block = 0; block < 2; ++block) {
      uint32_t w[4];
      stream_words(seed, replica, step, (uint32_t)i, ORA_TAG_XI, block, w);
      double u1 = u53(w[0], w[1]);
      double u2 = u53(w[2], w[3]);
      double rad = sqrt(-2.0 * log(u1));
      double th = two_pi * u2;
      if (block == 0) {
        xi[3 * i + 0] = rad * cos(th);
        xi[3 * i + 1] = rad * sin(th);
      } else {
        xi[3 * i + 2] = rad * cos(th);
      }
    }
  }
}

/* ------------------------------------------------------------------------ */
/* System and potentials                                                     */
/* ------------------------------------------------------------------------ */
typedef struct {
  int n;              /* atoms */
  double L;           /* cubic box edge */
  const double *mass; /* [n] */
  double dt, gamma, kT, fu;
} ora_sys;

enum { ORA_POT_NONE = 0, ORA_POT_LJ = 1, ORA_POT_HARMONIC = 2, ORA_POT_EXT = 3 };

/* A force field defined in another oracle file (the message-passing target,
 * the pair and learned drafts): energy returned, forces written to F[n][3]. */
typedef double (*ora_ext_fn)(const void *ctx, int n, const double *x, double L, double *F);

typedef struct {
  int kind;
  double rc;             /* Lennard-Jones cutoff */
  double eps, sig;       /* Lennard-Jones epsilon, sigma */
  double k;              /* harmonic tether stiffness */
  const double *qref;    /* tether anchors [n][3] */
  const double *offset;  /* optional additive force field b [n][3] (test drafts) */
  ora_ext_fn ext;        /* ORA_POT_EXT: the force field and its context */
  const void *ext_ctx;
} ora_pot;

/* wrap one coordinate into [0, L); returns the image shift applied */
static int wrap1(double *x, double L) {
  double f = floor(*x / L);
  *x = *x - f * L;
  int s = (int)f;
  if (*x >= L) { *x -= L; s += 1; }
  if (*x < 0.0) { *x += L; s -= 1; }
  return s;
}

/* ------------------------------------------------------------------------ */
/* Pair enumeration.  The set is every ordered (i, j, image n) with          */
/*   |q_j + n L - q_i| < r_c,  (j, n) != (i, 0),                            */
/* evaluated in binary64 as dx = (x_j - x_i) + n_x L, d2 = (dx dx + dy dy)   */
/* + dz dz, test d2 < r_c * r_c.                                             */
/* ------------------------------------------------------------------------ */
static inline int pair_inside(const double *xi, const double *xj, int nx,
                              int ny, int nz, double L, double rc2,
                              double d[3], double *d2) {
  d[0] = (xj[0] - xi[0]) + (double)nx * L;
  d[1] = (xj[1] - xi[1]) + (double)ny * L;
  d[2] = (xj[2] - xi[2]) + (double)nz * L;
  *d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  return *d2 < rc2;
}

/* Brute force over all j and all images |n_a| <= ceil(rc / L).  Writes up to
 * `cap` records (i, j, nx, ny, nz) and returns the total count. */
long ora_pairs_brute(int n, const double *x, double L, double rc,
                     int32_t *out, long cap) {
  int nmax = (int)ceil(rc / L);
  double rc2 = rc * rc;
  long cnt = 0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      for (int nx = -nmax; nx <= nmax; ++nx)
        for (int ny = -nmax; ny <= nmax; ++ny)
          for (int nz = -nmax; nz <= nmax; ++nz) {
            if (j == i && nx == 0 && ny == 0 && nz == 0) continue;
            double d[3], d2;
            if (!pair_inside(&x[3 * i], &x[3 * j], nx, ny, nz, L, rc2, d, &d2))
              continue;
            if (cnt < cap) {
              int32_t *r = &out[5 * cnt];
              r[0] = i; r[1] = j; r[2] = nx; r[3] = ny; r[4] = nz;
            }
            ++cnt;
          }
  return cnt;
}

/* Linked-cell enumeration (requires floor(L / rc) >= 3 so that each image
 * within rc lies in one of the 27 neighbouring cells exactly once). */
typedef struct {
  int nc;
  int *head; /* [nc^3] */
  int *next; /* [n] */
} cells_t;

static int cells_build(cells_t *c, int n, const double *x, double L,
                       double rc) {
  int nc = (int)floor(L / rc);
  if (nc < 3) return 0;
  c->nc = nc;
  c->head = (int *)malloc(sizeof(int) * (size_t)nc * nc * nc);
  c->next = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  for (int a = 0; a < nc * nc * nc; ++a) c->head[a] = -1;
  for (int i = n - 1; i >= 0; --i) { /* head-insert in reverse: ascending lists */
    int ci[3];
    for (int d = 0; d < 3; ++d) {
      int v = (int)floor(x[3 * i + d] / L * nc);
      if (v < 0) v = 0;
      if (v >= nc) v = nc - 1;
      ci[d] = v;
    }
    int id = ci[0] + nc * (ci[1] + nc * ci[2]);
    c->next[i] = c->head[id];
    c->head[id] = i;
  }
  return 1;
}

static void cells_free(cells_t *c) {
  free(c->head);
  free(c->next);
}

static int cell_of(const double *xi, double L, int nc, int d) {
  int v = (int)floor(xi[d] / L * nc);
  if (v < 0) v = 0;
  if (v >= nc) v = nc - 1;
  return v;
}

long ora_pairs_cells(int n, const double *x, double L, double rc,
                     int32_t *out, long cap) {
  cells_t c;
  if (!cells_build(&c, n, x, L, rc)) return -1;
  int nc = c.nc;
  double rc2 = rc * rc;
  long cnt = 0;
  for (int i = 0; i < n; ++i) {
    int cx = cell_of(&x[3 * i], L, nc, 0), cy = cell_of(&x[3 * i], L, nc, 1),
        cz = cell_of(&x[3 * i], L, nc, 2);
    for (int oz = -1; oz <= 1; ++oz)
      for (int oy = -1; oy <= 1; ++oy)
        for (int ox = -1; ox <= 1; ++ox) {
          int tx = cx + ox, ty = cy + oy, tz = cz + oz;
          int nx = 0, ny = 0, nz = 0;
          if (tx < 0) { tx += nc; nx = -1; } else if (tx >= nc) { tx -= nc; nx = 1; }
          if (ty < 0) { ty += nc; ny = -1; } else if (ty >= nc) { ty -= nc; ny = 1; }
          if (tz < 0) { tz += nc; nz = -1; } else if (tz >= nc) { tz -= nc; nz = 1; }
          for (int j = c.head[tx + nc * (ty + nc * tz)]; j >= 0; j = c.next[j]) {
            if (j == i && nx == 0 && ny == 0 && nz == 0) continue;
            double d[3], d2;
            if (!pair_inside(&x[3 * i], &x[3 * j], nx, ny, nz, L, rc2, d, &d2))
              continue;
            if (cnt < cap) {
              int32_t *r = &out[5 * cnt];
              r[0] = i; r[1] = j; r[2] = nx; r[3] = ny; r[4] = nz;
            }
            ++cnt;
          }
        }
  }
  cells_free(&c);
  return cnt;
}

/* ------------------------------------------------------------------------ */
/* Potentials: energy U(q) and forces F = -dU/dq (Sec. 2.1)                  */
/* ------------------------------------------------------------------------ */

/* Truncated and energy-shifted Lennard-Jones pair energy (reading fixed for
 * this implementation; the paper's force fields are external models):
 *   phi(r) = 4 eps [(sig/r)^12 - (sig/r)^6] - 4 eps [(sig/rc)^12 - (sig/rc)^6]
 * for r < rc, 0 otherwise.  Returns phi(r) and writes phi'(r). */
static double lj_phi(double r, double eps, double sig, double rc,
                     double *dphi) {
  double sr = sig / r, src = sig / rc;
  double sr6 = sr * sr * sr * sr * sr * sr;
  double src6 = src * src * src * src * src * src;
  *dphi = 4.0 * eps * (-12.0 * sr6 * sr6 + 6.0 * sr6) / r;
  return 4.0 * eps * (sr6 * sr6 - sr6) - 4.0 * eps * (src6 * src6 - src6);
}

/* Force on atom i from the pair record at separation d = q_j + nL - q_i:
 * F_i = -dphi/dq_i = phi'(r) d / r; each ordered record contributes half of
 * the pair energy. */
static double lj_atom(int i, int n, const double *x, double L,
                      const ora_pot *P, const cells_t *c, double Fi[3]) {
  double rc2 = P->rc * P->rc, e = 0.0;
  Fi[0] = Fi[1] = Fi[2] = 0.0;
  if (c) {
    int nc = c->nc;
    int cx = cell_of(&x[3 * i], L, nc, 0), cy = cell_of(&x[3 * i], L, nc, 1),
        cz = cell_of(&x[3 * i], L, nc, 2);
    for (int oz = -1; oz <= 1; ++oz)
      for (int oy = -1; oy <= 1; ++oy)
        for (int ox = -1; ox <= 1; ++ox) {
          int tx = cx + ox, ty = cy + oy, tz = cz + oz;
          int nx = 0, ny = 0, nz = 0;
          if (tx < 0) { tx += nc; nx = -1; } else if (tx >= nc) { tx -= nc; nx = 1; }
          if (ty < 0) { ty += nc; ny = -1; } else if (ty >= nc) { ty -= nc; ny = 1; }
          if (tz < 0) { tz += nc; nz = -1; } else if (tz >= nc) { tz -= nc; nz = 1; }
          for (int j = c->head[tx + nc * (ty + nc * tz)]; j >= 0; j = c->next[j]) {
            if (j == i && nx == 0 && ny == 0 && nz == 0) continue;
            double d[3], d2;
            if (!pair_inside(&x[3 * i], &x[3 * j], nx, ny, nz, L, rc2, d, &d2))
              continue;
            double r = sqrt(d2), dphi;
            e += 0.5 * lj_phi(r, P->eps, P->sig, P->rc, &dphi);
            for (int a = 0; a < 3; ++a) Fi[a] += dphi * d[a] / r;
          }
        }
  } else {
    int nmax = (int)ceil(P->rc / L);
    for (int j = 0; j < n; ++j)
      for (int nx = -nmax; nx <= nmax; ++nx)
        for (int ny = -nmax; ny <= nmax; ++ny)
          for (int nz = -nmax; nz <= nmax; ++nz) {
            if (j == i && nx == 0 && ny == 0 && nz == 0) continue;
            double d[3], d2;
            if (!pair_inside(&x[3 * i], &x[3 * j], nx, ny, nz, L, rc2, d, &d2))
              continue;
            double r = sqrt(d2), dphi;
            e += 0.5 * lj_phi(r, P->eps, P->sig, P->rc, &dphi);
            for (int a = 0; a < 3; ++a) Fi[a] += dphi * d[a] / r;
          }
  }
  return e;
}

/* Harmonic tether U = k/2 sum_i |q_i - qref_i|^2 (minimum-image difference). */
static double tether_atom(int i, const double *x, double L, const ora_pot *P,
                          double Fi[3]) {
  double e = 0.0;
  for (int a = 0; a < 3; ++a) {
    double d = x[3 * i + a] - P->qref[3 * i + a];
    d -= L * nearbyint(d / L);
    Fi[a] = -P->k * d;
    e += 0.5 * P->k * d * d;
  }
  return e;
}

/* Energy U(q) and forces F(q) for potential P.  `parallel` lets the atom
 * loop use OpenMP (callers inside a parallel region pass 0).  The per-atom
 * sums are independent of the thread count. */
double ora_energy_forces(const ora_pot *P, int n, const double *x, double L,
                         double *F, int parallel) {
  if (P->kind == ORA_POT_EXT) {
    double E = P->ext(P->ext_ctx, n, x, L, F);
    if (P->offset)
      for (int c = 0; c < 3 * n; ++c) F[c] += P->offset[c];
    return E;
  }
  cells_t cells, *cp = NULL;
  if (P->kind == ORA_POT_LJ && cells_build(&cells, n, x, L, P->rc)) cp = &cells;
  double *e_atom = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
#pragma omp parallel for schedule(static) if (parallel && n > 256)
  for (int i = 0; i < n; ++i) {
    double Fi[3] = {0.0, 0.0, 0.0}, e = 0.0;
    if (P->kind == ORA_POT_LJ) e = lj_atom(i, n, x, L, P, cp, Fi);
    else if (P->kind == ORA_POT_HARMONIC) e = tether_atom(i, x, L, P, Fi);
    if (P->offset)
      for (int a = 0; a < 3; ++a) Fi[a] += P->offset[3 * i + a];
    for (int a = 0; a < 3; ++a) F[3 * i + a] = Fi[a];
    e_atom[i] = e;
  }
  double E = 0.0;
  for (int i = 0; i < n; ++i) E += e_atom[i];
  free(e_atom);
  if (cp) cells_free(cp);
  return E;
}

/* ------------------------------------------------------------------------ */
/* Integrator pieces (Eq. aboba; Eq. bob)                                    */
/* ------------------------------------------------------------------------ */

/* (A): q <- q + dt/2 M^-1 p, then wrap into the box. */
static void step_A(const ora_sys *S, const double *p, double *q,
                   int32_t *img) {
  for (int i = 0; i < S->n; ++i)
    for (int a = 0; a < 3; ++a) {
      q[3 * i + a] = q[3 * i + a] + (0.5 * S->dt) * p[3 * i + a] / S->mass[i];
      int s = wrap1(&q[3 * i + a], S->L);
      if (img) img[3 * i + a] += s;
    }
}

/* Mean of the (BOB) Gaussian, Eq. bob:
 *   <p_n> = e^{-gamma dt} p_{n-1} + (1 + e^{-gamma dt}) dt/2 F_n   */
static void bob_mean(const ora_sys *S, const double *p_prev, const double *F,
                     double *mean) {
  double a = exp(-S->gamma * S->dt);
  for (int c = 0; c < 3 * S->n; ++c)
    mean[c] = a * p_prev[c] + (1.0 + a) * (0.5 * S->dt) * S->fu * F[c];
}

/* Square root of the diagonal covariance Sigma = M kT (1 - e^{-2 gamma dt}). */
static void bob_sigma(const ora_sys *S, double *sig) {
  for (int i = 0; i < S->n; ++i) {
    double s = sqrt(S->mass[i] * S->kT * S->fu *
                    (1.0 - exp(-2.0 * S->gamma * S->dt)));
    sig[3 * i] = sig[3 * i + 1] = sig[3 * i + 2] = s;
  }
}

/* One plain (ABOBA) step with forces of P and noise xi: A, then the (BOB)
 * Gaussian draw, then A.  Returns U at the midpoint positions. */
double ora_aboba_step(const ora_sys *S, const ora_pot *P, double *q, double *p,
                      int32_t *img, const double *xi) {
  int m = 3 * S->n;
  double *F = (double *)malloc(sizeof(double) * m);
  double *mu = (double *)malloc(sizeof(double) * m);
  double *sg = (double *)malloc(sizeof(double) * m);
  step_A(S, p, q, img);
  double E = ora_energy_forces(P, S->n, q, S->L, F, 1);
  bob_mean(S, p, F, mu);
  bob_sigma(S, sg);
  for (int c = 0; c < m; ++c) p[c] = mu[c] + sg[c] * xi[c];
  step_A(S, p, q, img);
  free(F); free(mu); free(sg);
  return E;
}

/* ------------------------------------------------------------------------ */
/* Transport map: reflection-maximal coupling, Eq. reflectionVerify          */
/* ------------------------------------------------------------------------ */

/* Given the target mean <p>, the draft mean <p~>, the diagonal sqrt(Sigma)
 * and the draft sample p~ (all length m), returns 1 and p_out = p~ if
 *   u <= min{1, N(p~; <p>, Sigma) / N(p~; <p~>, Sigma)},
 * else 0 and p_out = <p> + Sigma^{1/2} (I - 2 delta delta^T / delta^T delta) z
 * with z = Sigma^{-1/2}(p~ - <p~>) and delta = Sigma^{-1/2}(<p~> - <p>).
 * The log density ratio is evaluated from its definition (two Mahalanobis
 * norms).  S1 = delta.z and S2 = delta.delta are reported for inspection. */
int ora_reflection_verify(int m, const double *mu_t, const double *mu_d,
                          const double *sig, const double *pd, double u,
                          double *p_out, double *logr_out, double *S1_out,
                          double *S2_out) {
  double mt = 0.0, md = 0.0, s1 = 0.0, s2 = 0.0;
  for (int c = 0; c < m; ++c) {
    double wt = (pd[c] - mu_t[c]) / sig[c];
    double z = (pd[c] - mu_d[c]) / sig[c];
    double dl = (mu_d[c] - mu_t[c]) / sig[c];
    mt += wt * wt;
    md += z * z;
    s1 += dl * z;
    s2 += dl * dl;
  }
  double logr = -0.5 * mt + 0.5 * md;
  if (logr_out) *logr_out = logr;
  if (S1_out) *S1_out = s1;
  if (S2_out) *S2_out = s2;
  double ratio = exp(logr);
  int accept = u <= (ratio < 1.0 ? ratio : 1.0);
  if (accept) {
    if (p_out) memcpy(p_out, pd, sizeof(double) * m);
    return 1;
  }
  /* rejection: reflect z across the hyperplane normal to delta */
  double coef = 2.0 * s1 / s2;
  if (p_out)
    for (int c = 0; c < m; ++c) {
      double z = (pd[c] - mu_d[c]) / sig[c];
      double dl = (mu_d[c] - mu_t[c]) / sig[c];
      p_out[c] = mu_t[c] + sig[c] * (z - coef * dl);
    }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* LSD window (Alg. 1 with lookahead K, per-step maps of Alg. 2)             */
/* ------------------------------------------------------------------------ */
typedef struct {
  /* per frame k = 1..K (stored at k-1) */
  double *logr, *S1, *S2, *E_target;
  int8_t *accept;
  /* optional frame arrays (NULL to skip): [K][n][3], p_draft [K+1][n][3];
   * F_draft holds the bare draft forces (before any error correction) */
  double *q_mid, *p_draft, *F_draft, *F_target;
  int32_t n_committed; /* frames committed: first rejected index, else K */
  int32_t rejected;    /* 1 if the last committed frame was reflected */
} ora_window_out;

/* draft_step of Alg. 2: (q, p) = y is advanced in place to y'; the midpoint
 * positions (map f) and the bare draft forces F~ are returned.  With
 * speculative error correction (App. D, Alg. 3) the mean of the draft
 * Gaussian is taken from F~ + dF, dF being the cached target-minus-draft force
 * error of the last committed step, and F_c receives that corrected force;
 * without it (dF == NULL) F_c = F~.  Linear variant (dF_prev != NULL, the
 * error of the committed step before): the error is extrapolated to this
 * draft, which produces the (lag)-th step after the last committed one:
 * dF + lag (dF - dF_prev). */
static void draft_step(const ora_sys *S, const ora_pot *D, double *q,
                       double *p, int32_t *img, const double *xi,
                       double *q_mid, double *F_d, const double *dF,
                       const double *dF_prev, int lag, double *F_c) {
  int m = 3 * S->n;
  double *mu = (double *)malloc(sizeof(double) * m);
  double *sg = (double *)malloc(sizeof(double) * m);
  step_A(S, p, q, img);                           /* q~ <- q~ + dt/2 M^-1 p~ */
  memcpy(q_mid, q, sizeof(double) * m);
  ora_energy_forces(D, S->n, q, S->L, F_d, 1);    /* F~ <- draft forces */
  for (int c = 0; c < m; ++c) {
    double corr = dF ? dF[c] : 0.0;
    if (dF && dF_prev) corr = dF[c] + (double)lag * (dF[c] - dF_prev[c]);
    F_c[c] = F_d[c] + corr;
  }
  bob_mean(S, p, F_c, mu);                        /* <p~> from Eq. bob */
  bob_sigma(S, sg);
  for (int c = 0; c < m; ++c) p[c] = mu[c] + sg[c] * xi[c]; /* p~ ~ N */
  step_A(S, p, q, img);                           /* q~ <- q~ + dt/2 M^-1 p~ */
  free(mu); free(sg);
}

/* verify_step of Alg. 2 after map f: target forces at the midpoint q_mid,
 * target mean <p>, draft mean <p~> recomputed from F~, reflectionVerify on
 * the stored draft momentum p_new, then map g.  On return p_out / q_out hold
 * the verified state (equal to the draft state when accepted). */
int ora_verify_frame(const ora_sys *S, const ora_pot *T, const double *q_mid,
                     const double *p_prev, const double *p_new,
                     const double *F_d, double u, int parallel, double *F_t,
                     double *E_t, double *logr, double *S1, double *S2,
                     double *p_out, double *q_out) {
  int m = 3 * S->n;
  double *mu_t = (double *)malloc(sizeof(double) * m);
  double *mu_d = (double *)malloc(sizeof(double) * m);
  double *sg = (double *)malloc(sizeof(double) * m);
  double E = ora_energy_forces(T, S->n, q_mid, S->L, F_t, parallel);
  if (E_t) *E_t = E;
  bob_mean(S, p_prev, F_t, mu_t);
  bob_mean(S, p_prev, F_d, mu_d);
  bob_sigma(S, sg);
  int acc = ora_reflection_verify(m, mu_t, mu_d, sg, p_new, u, p_out, logr, S1,
                                  S2);
  if (q_out) {
    memcpy(q_out, q_mid, sizeof(double) * m);
    step_A(S, p_out, q_out, NULL); /* map g */
  }
  free(mu_t); free(mu_d); free(sg);
  return acc;
}

/* One synchronous window from the verified state (q, p, img): draft K steps
 * with noise xi[K][n][3], verify all K in parallel with uniforms u[K], keep
 * the prefix up to and including the first rejection (Alg. 1), and advance
 * (q, p, img) to the last kept state.  dF (NULL: no error correction) is the
 * error cache of App. D: every draft of the window is corrected by its value
 * on entry, and on return it holds F - F~ (target minus bare draft force) of
 * the last committed step, accepted or reflected.  Linear variant: dF_prev
 * holds the error of the committed step before and *samples the number of
 * committed errors seen (capped at 2); with two samples, draft k of the
 * window (producing the (k+1)-th new step) uses dF + (k+1) (dF - dF_prev). */
int ora_lsd_window(const ora_sys *S, const ora_pot *T, const ora_pot *D,
                   double *q, double *p, int32_t *img, int K,
                   const double *xi, const double *u, ora_window_out *out,
                   double *dF, double *dF_prev, int *samples) {
  int n = S->n, m = 3 * n;
  double *qm = (double *)malloc(sizeof(double) * (size_t)K * m);
  double *pd = (double *)malloc(sizeof(double) * (size_t)(K + 1) * m);
  double *Fd = (double *)malloc(sizeof(double) * (size_t)K * m);
  double *Fc = (double *)malloc(sizeof(double) * (size_t)K * m);
  double *Ft = (double *)malloc(sizeof(double) * (size_t)K * m);
  double *pv = (double *)malloc(sizeof(double) * (size_t)K * m);
  double *qv = (double *)malloc(sizeof(double) * (size_t)K * m);
  int32_t *imgs = (int32_t *)malloc(sizeof(int32_t) * (size_t)(K + 1) * m);
  double *qd = (double *)malloc(sizeof(double) * (size_t)(K + 1) * m);
  int8_t *acc = (int8_t *)malloc((size_t)K);
  double *lr = (double *)malloc(sizeof(double) * K);
  double *s1 = (double *)malloc(sizeof(double) * K);
  double *s2 = (double *)malloc(sizeof(double) * K);
  double *et = (double *)malloc(sizeof(double) * K);

  /* drafting: serial */
  memcpy(qd, q, sizeof(double) * m);
  memcpy(pd, p, sizeof(double) * m);
  memcpy(imgs, img, sizeof(int32_t) * m);
  for (int k = 0; k < K; ++k) {
    memcpy(&qd[(size_t)(k + 1) * m], &qd[(size_t)k * m], sizeof(double) * m);
    memcpy(&pd[(size_t)(k + 1) * m], &pd[(size_t)k * m], sizeof(double) * m);
    memcpy(&imgs[(size_t)(k + 1) * m], &imgs[(size_t)k * m], sizeof(int32_t) * m);
    draft_step(S, D, &qd[(size_t)(k + 1) * m], &pd[(size_t)(k + 1) * m],
               &imgs[(size_t)(k + 1) * m], &xi[(size_t)k * m],
               &qm[(size_t)k * m], &Fd[(size_t)k * m], dF,
               (dF_prev && samples && *samples >= 2) ? dF_prev : NULL, k + 1,
               &Fc[(size_t)k * m]);
  }
  /* verification: independent frames, in parallel */
#pragma omp parallel for schedule(dynamic, 1)
  for (int k = 0; k < K; ++k) {
    acc[k] = (int8_t)ora_verify_frame(
        S, T, &qm[(size_t)k * m], &pd[(size_t)k * m], &pd[(size_t)(k + 1) * m],
        &Fc[(size_t)k * m], u[k], 0, &Ft[(size_t)k * m], &et[k], &lr[k], &s1[k],
        &s2[k], &pv[(size_t)k * m], &qv[(size_t)k * m]);
  }
  /* first rejection l; keep steps 1..l (Alg. 1) */
  int j = K, rej = 0;
  for (int k = 0; k < K; ++k)
    if (!acc[k]) { j = k + 1; rej = 1; break; }
  if (rej) {
    memcpy(p, &pv[(size_t)(j - 1) * m], sizeof(double) * m);
    memcpy(q, &qv[(size_t)(j - 1) * m], sizeof(double) * m);
    /* image counters of the verified state: those of the midpoint plus the
     * wrap applied by map g */
    memcpy(img, &imgs[(size_t)(j - 1) * m], sizeof(int32_t) * m);
    double *qt = (double *)malloc(sizeof(double) * m);
    memcpy(qt, &qd[(size_t)(j - 1) * m], sizeof(double) * m);
    step_A(S, &pd[(size_t)(j - 1) * m], qt, img); /* back to the midpoint */
    step_A(S, p, qt, img);                        /* map g */
    free(qt);
  } else {
    memcpy(p, &pd[(size_t)K * m], sizeof(double) * m);
    memcpy(q, &qd[(size_t)K * m], sizeof(double) * m);
    memcpy(img, &imgs[(size_t)K * m], sizeof(int32_t) * m);
  }
  if (dF) { /* new error caches from the EC-uncorrected draft forces */
    for (int c = 0; c < m; ++c) {
      if (dF_prev)
        dF_prev[c] = j >= 2 ? Ft[(size_t)(j - 2) * m + c] - Fd[(size_t)(j - 2) * m + c] : dF[c];
      dF[c] = Ft[(size_t)(j - 1) * m + c] - Fd[(size_t)(j - 1) * m + c];
    }
    if (samples) *samples = (*samples + j) < 2 ? (*samples + j) : 2;
  }
  if (out) {
    if (out->logr) memcpy(out->logr, lr, sizeof(double) * K);
    if (out->S1) memcpy(out->S1, s1, sizeof(double) * K);
    if (out->S2) memcpy(out->S2, s2, sizeof(double) * K);
    if (out->E_target) memcpy(out->E_target, et, sizeof(double) * K);
    if (out->accept) memcpy(out->accept, acc, (size_t)K);
    if (out->q_mid) memcpy(out->q_mid, qm, sizeof(double) * (size_t)K * m);
    if (out->p_draft) memcpy(out->p_draft, pd, sizeof(double) * (size_t)(K + 1) * m);
    if (out->F_draft) memcpy(out->F_draft, Fd, sizeof(double) * (size_t)K * m);
    if (out->F_target) memcpy(out->F_target, Ft, sizeof(double) * (size_t)K * m);
    out->n_committed = j;
    out->rejected = rej;
  }
  free(qm); free(pd); free(Fd); free(Fc); free(Ft); free(pv); free(qv); free(imgs);
  free(qd); free(acc); free(lr); free(s1); free(s2); free(et);
  return j;
}

/* ------------------------------------------------------------------------ */
/* Runs with the step-keyed Philox stream                                    */
/* ------------------------------------------------------------------------ */
typedef struct {
  int64_t windows;      /* windows executed */
  int64_t rejections;   /* windows ending in a rejection */
  int64_t frames;       /* frames drafted and verified */
  int64_t committed;    /* steps committed */
} ora_run_stats;

/* LSD from committed step `step0` until `n_steps` more steps are committed,
 * in windows of at most K frames.  Optionally records the committed states
 * traj_q / traj_p [n_steps][n][3] (NULL to skip). */
void ora_lsd_run(const ora_sys *S, const ora_pot *T, const ora_pot *D,
                 double *q, double *p, int32_t *img, uint64_t seed,
                 uint32_t replica, uint64_t step0, int64_t n_steps, int K,
                 double *traj_q, double *traj_p, ora_run_stats *st, double *dF,
                 double *dF_prev) {
  int samples = 0; /* committed errors held by the linear error correction */
  int n = S->n, m = 3 * n;
  double *xi = (double *)malloc(sizeof(double) * (size_t)K * m);
  double *u = (double *)malloc(sizeof(double) * K);
  int8_t *acc = (int8_t *)malloc((size_t)K);
  double *qm = traj_q ? (double *)malloc(sizeof(double) * (size_t)K * m) : NULL;
  double *pd = traj_q ? (double *)malloc(sizeof(double) * (size_t)(K + 1) * m) : NULL;
  int32_t *im = traj_q ? (int32_t *)malloc(sizeof(int32_t) * m) : NULL;
  ora_run_stats s = {0, 0, 0, 0};
  int64_t done = 0;
  while (done < n_steps) {
    int Kw = K;
    if ((int64_t)Kw > n_steps - done) Kw = (int)(n_steps - done);
    uint64_t base = step0 + (uint64_t)done;
    for (int k = 0; k < Kw; ++k) {
      ora_normals(seed, replica, base + (uint64_t)k + 1u, n, &xi[(size_t)k * m]);
      u[k] = ora_uniform(seed, replica, base + (uint64_t)k + 1u);
    }
    ora_window_out o;
    memset(&o, 0, sizeof(o));
    o.accept = acc;
    o.q_mid = qm;
    o.p_draft = pd;
    int j = ora_lsd_window(S, T, D, q, p, img, Kw, xi, u, &o, dF, dF_prev, &samples);
    if (traj_q) {
      /* committed states: accepted draft states then the final state */
      double *qt = (double *)malloc(sizeof(double) * m);
      for (int k = 0; k < j - 1; ++k) {
        memcpy(qt, &qm[(size_t)k * m], sizeof(double) * m);
        memset(im, 0, sizeof(int32_t) * m);
        step_A(S, &pd[(size_t)(k + 1) * m], qt, im);
        memcpy(&traj_q[(size_t)(done + k) * m], qt, sizeof(double) * m);
        memcpy(&traj_p[(size_t)(done + k) * m], &pd[(size_t)(k + 1) * m],
               sizeof(double) * m);
      }
      memcpy(&traj_q[(size_t)(done + j - 1) * m], q, sizeof(double) * m);
      memcpy(&traj_p[(size_t)(done + j - 1) * m], p, sizeof(double) * m);
      free(qt);
    }
    s.windows += 1;
    s.rejections += o.rejected;
    s.frames += Kw;
    s.committed += j;
    done += j;
  }
  if (st) *st = s;
  free(xi); free(u); free(acc);
  if (qm) free(qm);
  if (pd) free(pd);
  if (im) free(im);
}

/* Plain target Langevin (ABOBA with target forces) for n_steps steps with the
 * same step-keyed stream; optional trajectory recording as above. */
void ora_plain_run(const ora_sys *S, const ora_pot *T, double *q, double *p,
                   int32_t *img, uint64_t seed, uint32_t replica,
                   uint64_t step0, int64_t n_steps, double *traj_q,
                   double *traj_p, double *energies) {
  int m = 3 * S->n;
  double *xi = (double *)malloc(sizeof(double) * m);
  for (int64_t t = 0; t < n_steps; ++t) {
    ora_normals(seed, replica, step0 + (uint64_t)t + 1u, S->n, xi);
    double E = ora_aboba_step(S, T, q, p, img, xi);
    if (energies) energies[t] = E;
    if (traj_q) memcpy(&traj_q[(size_t)t * m], q, sizeof(double) * m);
    if (traj_p) memcpy(&traj_p[(size_t)t * m], p, sizeof(double) * m);
  }
  free(xi);
}

/* Kinetic energy of one system in binary64: the sum over atoms i and axes
 * d of p_id^2 / (2 m_i), with p row-major [n][3] and m per atom.  This is
 * the observable behind the kinetic temperature of Sec. 4.3 (Tab. heating),
 * T_kin = 2 K / (3 n k_B) (the paper prints the formula without the 3; see
 * the reading in the Python wrapper).  Summed serially in atom order. */
double ora_kinetic_energy(int n, const double *p, const double *mass) {
  double k = 0.0;
  for (int i = 0; i < n; ++i)
    for (int d = 0; d < 3; ++d) k += p[3 * i + d] * p[3 * i + d] / (2.0 * mass[i]);
  return k;
}

int ora_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* (OBABO) splitting (App. E)                                                */
/* ------------------------------------------------------------------------ */
/* Normals of the stream with an explicit tag (same layout as ora_normals).
 * Tag 3 draws the extra noise of the (OBABO) outputs: the initial (O) half
 * step at step 0 and the conditional half-step noise of step n. */
#define ORA_TAG_OB 3u
void ora_normals_tag(uint64_t seed, uint32_t replica, uint64_t step, uint32_t tag, int n,
                     double *xi) {
  const double two_pi = 6.283185307179586476925286766559;
  for (int i = 0; i < n; ++i) {
    for (uint32_t block = 0; block < 2; ++block) {
      uint32_t w[4];
      stream_words(seed, replica, step, (uint32_t)i, tag, block, w);
      double rad = sqrt(-2.0 * log(u53(w[0], w[1])));
      double th = two_pi * u53(w[2], w[3]);
      if (block == 0) {
        xi[3 * i + 0] = rad * cos(th);
        xi[3 * i + 1] = rad * sin(th);
      } else {
        xi[3 * i + 2] = rad * cos(th);
      }
    }
  }
}

/* sqrt of the half-step (O) covariance Sigma_1/2 = M kT (1 - e^{-gamma dt}) */
static double half_sigma(const ora_sys *S, int i) {
  return sqrt(S->mass[i] * S->kT * S->fu * (1.0 - exp(-S->gamma * S->dt)));
}

/* One plain (OBABO) step (Eq. obabo): O(dt/2) with xi1, B(dt/2), A(dt),
 * B(dt/2), O(dt/2) with xi2.  Returns U at the new positions. */
double ora_obabo_step(const ora_sys *S, const ora_pot *P, double *q, double *p, int32_t *img,
                      const double *xi1, const double *xi2) {
  int m = 3 * S->n;
  double *F = (double *)malloc(sizeof(double) * m);
  double ah = exp(-0.5 * S->gamma * S->dt);
  for (int c = 0; c < m; ++c) p[c] = ah * p[c] + half_sigma(S, c / 3) * xi1[c];   /* O */
  ora_energy_forces(P, S->n, q, S->L, F, 1);
  for (int c = 0; c < m; ++c) p[c] += 0.5 * S->dt * S->fu * F[c];                  /* B */
  for (int i = 0; i < S->n; ++i)                                                   /* A */
    for (int a = 0; a < 3; ++a) {
      q[3 * i + a] += S->dt * p[3 * i + a] / S->mass[i];
      int s = wrap1(&q[3 * i + a], S->L);
      if (img) img[3 * i + a] += s;
    }
  double E = ora_energy_forces(P, S->n, q, S->L, F, 1);
  for (int c = 0; c < m; ++c) p[c] += 0.5 * S->dt * S->fu * F[c];                  /* B */
  for (int c = 0; c < m; ++c) p[c] = ah * p[c] + half_sigma(S, c / 3) * xi2[c];    /* O */
  free(F);
  return E;
}

/* n_steps plain (OBABO) steps; the two noises of step t come from tags 1 and
 * 3 of the stream at step step0 + t + 1. */
void ora_obabo_plain_run(const ora_sys *S, const ora_pot *P, double *q, double *p, int32_t *img,
                         uint64_t seed, uint32_t replica, uint64_t step0, int64_t n_steps) {
  int m = 3 * S->n;
  double *x1 = (double *)malloc(sizeof(double) * m);
  double *x2 = (double *)malloc(sizeof(double) * m);
  for (int64_t t = 0; t < n_steps; ++t) {
    uint64_t s = step0 + (uint64_t)t + 1u;
    ora_normals_tag(seed, replica, s, ORA_TAG_OB, S->n, x1);
    ora_normals(seed, replica, s, S->n, x2);
    ora_obabo_step(S, P, q, p, img, x1, x2);
  }
  free(x1); free(x2);
}

/* Start of LSD for (OBABO) in the staggered frame (App. E): from the (OBABO)
 * state y_0 = (q, p), ybar_0 = OB(y_0) is an (O) half step with noise from
 * tag 3 at step `step`, then a (B) half step with the target force at q_0;
 * (q, p, img) become the (ABOBA) state whose next midpoint is
 * q_0 + dt pbar_0 / m (the staggered chain ybar_n = BOB(A(ybar_{n-1})) is the
 * (ABOBA) chain read at its midpoints). */
void ora_obabo_begin(const ora_sys *S, const ora_pot *T, double *q, double *p, int32_t *img,
                     uint64_t seed, uint32_t replica, uint64_t step) {
  int n = S->n, m = 3 * n;
  double *F = (double *)malloc(sizeof(double) * m);
  double *xi = (double *)malloc(sizeof(double) * m);
  double ah = exp(-0.5 * S->gamma * S->dt);
  ora_normals_tag(seed, replica, step, ORA_TAG_OB, n, xi);
  ora_energy_forces(T, n, q, S->L, F, 1);
  for (int c = 0; c < m; ++c)
    p[c] = ah * p[c] + half_sigma(S, c / 3) * xi[c] + 0.5 * S->dt * S->fu * F[c];
  step_A(S, p, q, img);
  free(F); free(xi);
}

/* The (OBABO) state y_n of committed step n from the staggered (ABOBA) state
 * (q, p) = (q_n + dt/2 pbar_n / m, pbar_n) and pbar_{n-1} = pprev:
 *   q_n  = the midpoint (back by a half step, wrapped),
 *   p_n  = e^{-gamma dt/2}(pbar_{n-1} + dt/2 F_n) + Sigma_1/2^{1/2} xi1*,
 * xi1* drawn from the Gaussian conditional on
 *   w = Sigma_1/2^{-1/2}(pbar_n - e^{-gamma dt} pbar_{n-1} - (1 + e^{-gamma dt}) dt/2 F_n):
 * mean e^{-gamma dt/2} w / (1 + e^{-gamma dt}), variance 1 / (1 + e^{-gamma dt}),
 * with noise from tag 3 at step n (Eq. obabo_conditional).  Writes
 * (q_out, p_out); img (may be NULL) receives the wrap of q_n. */
void ora_obabo_recover(const ora_sys *S, const ora_pot *T, const double *q, const double *p,
                       const double *pprev, uint64_t seed, uint32_t replica, uint64_t step,
                       double *q_out, double *p_out, int32_t *img) {
  int n = S->n, m = 3 * n;
  double *F = (double *)malloc(sizeof(double) * m);
  double *xi = (double *)malloc(sizeof(double) * m);
  double ah = exp(-0.5 * S->gamma * S->dt), a = exp(-S->gamma * S->dt);
  for (int i = 0; i < n; ++i)
    for (int d = 0; d < 3; ++d) {
      q_out[3 * i + d] = q[3 * i + d] - (0.5 * S->dt) * p[3 * i + d] / S->mass[i];
      int s = wrap1(&q_out[3 * i + d], S->L);
      if (img) img[3 * i + d] += s;
    }
  ora_energy_forces(T, n, q_out, S->L, F, 1);
  ora_normals_tag(seed, replica, step, ORA_TAG_OB, n, xi);
  double cw = ah / (1.0 + a), cs = 1.0 / sqrt(1.0 + a);
  for (int c = 0; c < m; ++c) {
    double sh = half_sigma(S, c / 3);
    double half_kick = 0.5 * S->dt * S->fu * F[c];
    double w = (p[c] - a * pprev[c] - (1.0 + a) * half_kick) / sh;
    double x1 = cw * w + cs * xi[c];
    p_out[c] = ah * (pprev[c] + half_kick) + sh * x1;
  }
  free(F); free(xi);
}

/* LSD for (OBABO) in the staggered frame (App. E), from the (OBABO) state
 * y_0 = (q, p) at step 0 to y_{n_steps}, returned in (q, p, img): the start
 * ybar_0 = OB(y_0) (ora_obabo_begin), (ABOBA) LSD windows on the staggered
 * state, and the recovery of y_n at the last committed step
 * (ora_obabo_recover). */
void ora_obabo_lsd_run(const ora_sys *S, const ora_pot *T, const ora_pot *D, double *q,
                       double *p, int32_t *img, uint64_t seed, uint32_t replica,
                       int64_t n_steps, int K, ora_run_stats *st) {
  int n = S->n, m = 3 * n;
  double *xi = (double *)malloc(sizeof(double) * (size_t)K * m);
  double *u = (double *)malloc(sizeof(double) * K);
  double *pd = (double *)malloc(sizeof(double) * (size_t)(K + 1) * m);
  double *pprev = (double *)malloc(sizeof(double) * m);
  double *qs = (double *)malloc(sizeof(double) * m);
  double *ps = (double *)malloc(sizeof(double) * m);
  ora_obabo_begin(S, T, q, p, img, seed, replica, 0u);
  memcpy(pprev, p, sizeof(double) * m);
  if (st) memset(st, 0, sizeof(*st));
  int64_t done = 0;
  while (done < n_steps) {
    int Kw = (int)((n_steps - done) < K ? (n_steps - done) : K);
    for (int k = 0; k < Kw; ++k) {
      ora_normals(seed, replica, (uint64_t)done + (uint64_t)k + 1u, n, &xi[(size_t)k * m]);
      u[k] = ora_uniform(seed, replica, (uint64_t)done + (uint64_t)k + 1u);
    }
    ora_window_out o;
    memset(&o, 0, sizeof(o));
    o.p_draft = pd;
    int j = ora_lsd_window(S, T, D, q, p, img, Kw, xi, u, &o, NULL, NULL, NULL);
    memcpy(pprev, &pd[(size_t)(j - 1) * m], sizeof(double) * m); /* pbar_{n-1} */
    done += j;
    if (st) {
      st->windows += 1;
      st->committed += j;
      st->rejections += o.rejected;
      st->frames += Kw;
    }
  }
  memcpy(qs, q, sizeof(double) * m);
  memcpy(ps, p, sizeof(double) * m);
  ora_obabo_recover(S, T, qs, ps, pprev, seed, replica, (uint64_t)n_steps, q, p, img);
  free(xi); free(u); free(pd); free(pprev); free(qs); free(ps);
}
