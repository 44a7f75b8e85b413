/*
 * mpnn_oracle.c -- plain FP64 message-passing potential and its forces.
 *
 * TEST INFRASTRUCTURE ONLY (see lsd_oracle.c).  The paper's target force
 * fields are external interatomic potentials; the stand-in defined here is a
 * random-init message-passing network (reading fixed for this
 * implementation, see the design notes):
 *
 *   radial basis   e_b(r) = sqrt(2/rc) sin(b pi r / rc) / r,  b = 1..R
 *   cutoff         f_c(r) = (cos(pi r / rc) + 1) / 2           (r < rc)
 *   embedding      h0_i = W_emb[s_i]
 *   layer t        W_ij = f_c(r_ij) (A2 silu(A1 e(r_ij) + a1) + a2)
 *                  m_i  = sum_j W_ij (.) (B h_j)
 *                  h_i <- h_i + C2 silu(C1 m_i + c1) + c2
 *   readout        E = s_E sum_i (w2 . silu(W1 h_i + b1) + b2)
 *   forces         F = -dE/dq   (Sec. 2.1), by reverse-mode differentiation
 *                  written out below, layer by layer.
 *
 * Pairs are every ordered (i, j, image n) with |q_j + n L - q_i| < rc,
 * (j, n) != (i, 0), the same set the LJ oracle enumerates.  Weights come in
 * one flat vector in the order documented in mpnn_layout(); matrices are
 * stored [out][in].  Everything is evaluated in binary64 with plain loops.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

long ora_pairs_brute(int n, const double *x, double L, double rc, int32_t *out, long cap);
long ora_pairs_cells(int n, const double *x, double L, double rc, int32_t *out, long cap);

typedef struct {
  int n_species, H, R, T, RH;
  double rc;
  double scale; /* s_E */
  const double *w; /* flat weights */
} ora_mpnn;

typedef struct {
  const double *W_emb;
  const double *A1[8], *a1[8], *A2[8], *a2[8], *B[8], *C1[8], *c1[8], *C2[8], *c2[8];
  const double *W1, *b1, *w2, *b2;
} mpnn_view;

/* flat layout: W_emb [S][H]; per layer: A1 [H][R], a1 [H], A2 [H][H],
 * a2 [H], B [H][H], C1 [H][H], c1 [H], C2 [H][H], c2 [H]; then W1 [RH][H],
 * b1 [RH], w2 [RH], b2 [1].  Returns the total length. */
long ora_mpnn_layout(int S, int H, int R, int T, int RH) {
  long n = (long)S * H;
  n += (long)T * ((long)H * R + H + (long)H * H + H + (long)H * H + (long)H * H + H +
                  (long)H * H + H);
  n += (long)RH * H + RH + RH + 1;
  return n;
}

static void view(const ora_mpnn *M, mpnn_view *v) {
  const double *p = M->w;
  int H = M->H, R = M->R;
  v->W_emb = p; p += (long)M->n_species * H;
  for (int t = 0; t < M->T; ++t) {
    v->A1[t] = p; p += (long)H * R;
    v->a1[t] = p; p += H;
    v->A2[t] = p; p += (long)H * H;
    v->a2[t] = p; p += H;
    v->B[t] = p; p += (long)H * H;
    v->C1[t] = p; p += (long)H * H;
    v->c1[t] = p; p += H;
    v->C2[t] = p; p += (long)H * H;
    v->c2[t] = p; p += H;
  }
  v->W1 = p; p += (long)M->RH * H;
  v->b1 = p; p += M->RH;
  v->w2 = p; p += M->RH;
  v->b2 = p;
}

static double sigm(double x) { return 1.0 / (1.0 + exp(-x)); }
static double silu(double x) { return x * sigm(x); }
static double dsilu(double x) {
  double s = sigm(x);
  return s * (1.0 + x * (1.0 - s));
}

/* y[o] = sum_i A[o][i] x[i] (+ b[o]) */
static void matvec(const double *A, const double *b, const double *x, int nout, int nin,
                   double *y) {
  for (int o = 0; o < nout; ++o) {
    double s = b ? b[o] : 0.0;
    for (int i = 0; i < nin; ++i) s += A[(long)o * nin + i] * x[i];
    y[o] = s;
  }
}

/* y[i] += sum_o A[o][i] g[o]  (transposed product) */
static void matvec_t_acc(const double *A, const double *g, int nout, int nin, double *y) {
  for (int o = 0; o < nout; ++o)
    for (int i = 0; i < nin; ++i) y[i] += A[(long)o * nin + i] * g[o];
}

/* radial basis, cutoff and their r-derivatives */
static void radial(const ora_mpnn *M, double r, double *e, double *de, double *fc, double *dfc) {
  const double pi = 3.141592653589793238462643383279502884;
  double pre = sqrt(2.0 / M->rc);
  for (int b = 1; b <= M->R; ++b) {
    double k = b * pi / M->rc;
    e[b - 1] = pre * sin(k * r) / r;
    de[b - 1] = pre * (k * cos(k * r) / r - sin(k * r) / (r * r));
  }
  *fc = 0.5 * (cos(pi * r / M->rc) + 1.0);
  *dfc = -0.5 * (pi / M->rc) * sin(pi * r / M->rc);
}

/* Filter of layer t for one pair: W = f_c (A2 silu(A1 e + a1) + a2) and,
 * if dW != NULL, dW/dr. */
static void filter(const ora_mpnn *M, const mpnn_view *v, int t, const double *e,
                   const double *de, double fc, double dfc, double *W, double *dW) {
  int H = M->H, R = M->R;
  double *w = (double *)malloc(sizeof(double) * H);
  double *s = (double *)malloc(sizeof(double) * H);
  double *z = (double *)malloc(sizeof(double) * H);
  matvec(v->A1[t], v->a1[t], e, H, R, w);     /* w = A1 e + a1 */
  for (int c = 0; c < H; ++c) s[c] = silu(w[c]);
  matvec(v->A2[t], v->a2[t], s, H, H, z);     /* z = A2 s + a2 */
  for (int c = 0; c < H; ++c) W[c] = fc * z[c];
  if (dW) {
    double *dw = (double *)malloc(sizeof(double) * H);
    double *ds = (double *)malloc(sizeof(double) * H);
    double *dz = (double *)malloc(sizeof(double) * H);
    matvec(v->A1[t], NULL, de, H, R, dw);     /* dw/dr = A1 de/dr */
    for (int c = 0; c < H; ++c) ds[c] = dsilu(w[c]) * dw[c];
    matvec(v->A2[t], NULL, ds, H, H, dz);     /* dz/dr = A2 ds/dr */
    for (int c = 0; c < H; ++c) dW[c] = dfc * z[c] + fc * dz[c];
    free(dw); free(ds); free(dz);
  }
  free(w); free(s); free(z);
}

/* Filters of layer t for the pairs [k0, k1) into W[k - k0][H] (and dW): each
 * pair's filter is a function of its own distance only, so they are formed
 * side by side (in parallel) before the serial sums that use them. */
#define ORA_FILTER_CHUNK 16384
static void filter_chunk(const ora_mpnn *M, const mpnn_view *v, int t, long k0, long k1,
                         const double *e, const double *de, const double *fc,
                         const double *dfc, double *W, double *dW) {
  const int H = M->H, R = M->R;
#pragma omp parallel for schedule(static)
  for (long k = k0; k < k1; ++k)
    filter(M, v, t, &e[(size_t)k * R], &de[(size_t)k * R], fc[k], dfc[k],
           &W[(size_t)(k - k0) * H], dW ? &dW[(size_t)(k - k0) * H] : NULL);
}

/* Energy and forces (F may be NULL).  x [n][3] positions in a cubic box of
 * edge L; species [n].  Every sum runs serially in the order written; only
 * independent per-pair and per-atom products run in parallel. */
double ora_mpnn_energy_forces(const ora_mpnn *M, int n, const int32_t *species, const double *x,
                              double L, double *F) {
  mpnn_view v;
  view(M, &v);
  const int H = M->H, R = M->R, T = M->T, RH = M->RH;
  /* pair list */
  long np = (floor(L / M->rc) >= 3) ? ora_pairs_cells(n, x, L, M->rc, NULL, 0)
                                    : ora_pairs_brute(n, x, L, M->rc, NULL, 0);
  int32_t *P = (int32_t *)malloc(sizeof(int32_t) * 5 * (size_t)(np > 0 ? np : 1));
  if (floor(L / M->rc) >= 3) ora_pairs_cells(n, x, L, M->rc, P, np);
  else ora_pairs_brute(n, x, L, M->rc, P, np);
  double *d = (double *)malloc(sizeof(double) * 3 * (size_t)(np > 0 ? np : 1));
  double *r = (double *)malloc(sizeof(double) * (size_t)(np > 0 ? np : 1));
  double *e = (double *)malloc(sizeof(double) * (size_t)R * (np > 0 ? np : 1));
  double *de = (double *)malloc(sizeof(double) * (size_t)R * (np > 0 ? np : 1));
  double *fc = (double *)malloc(sizeof(double) * (size_t)(np > 0 ? np : 1));
  double *dfc = (double *)malloc(sizeof(double) * (size_t)(np > 0 ? np : 1));
  for (long k = 0; k < np; ++k) {
    int i = P[5 * k], j = P[5 * k + 1];
    for (int a = 0; a < 3; ++a)
      d[3 * k + a] = (x[3 * j + a] - x[3 * i + a]) + (double)P[5 * k + 2 + a] * L;
    r[k] = sqrt(d[3 * k] * d[3 * k] + d[3 * k + 1] * d[3 * k + 1] + d[3 * k + 2] * d[3 * k + 2]);
    radial(M, r[k], &e[(size_t)k * R], &de[(size_t)k * R], &fc[k], &dfc[k]);
  }
  const long chunk = ORA_FILTER_CHUNK;
  double *Wc = (double *)malloc(sizeof(double) * (size_t)chunk * H);
  double *dWc = (double *)malloc(sizeof(double) * (size_t)chunk * H);
  /* forward, keeping what the backward pass needs */
  double *h = (double *)malloc(sizeof(double) * (size_t)(T + 1) * n * H); /* h^0..h^T */
  double *xb = (double *)malloc(sizeof(double) * (size_t)T * n * H);     /* B h^{t-1} */
  double *u = (double *)malloc(sizeof(double) * (size_t)T * n * H);      /* C1 m + c1 */
  double *m = (double *)malloc(sizeof(double) * (size_t)n * H);
  for (int i = 0; i < n; ++i)
    memcpy(&h[(size_t)i * H], &v.W_emb[(size_t)species[i] * H], sizeof(double) * H);
  for (int t = 0; t < T; ++t) {
    const double *hp = &h[(size_t)t * n * H];
    double *hn = &h[(size_t)(t + 1) * n * H];
    double *xt = &xb[(size_t)t * n * H];
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) matvec(v.B[t], NULL, &hp[(size_t)i * H], H, H, &xt[(size_t)i * H]);
    memset(m, 0, sizeof(double) * (size_t)n * H);
    for (long k0 = 0; k0 < np; k0 += chunk) {
      long k1 = k0 + chunk < np ? k0 + chunk : np;
      filter_chunk(M, &v, t, k0, k1, e, de, fc, dfc, Wc, NULL);
      for (long k = k0; k < k1; ++k) {
        int i = P[5 * k], j = P[5 * k + 1];
        const double *Wf = &Wc[(size_t)(k - k0) * H];
        for (int c = 0; c < H; ++c) m[(size_t)i * H + c] += Wf[c] * xt[(size_t)j * H + c];
      }
    }
#pragma omp parallel
    {
      double *tmp = (double *)malloc(sizeof(double) * H);
#pragma omp for schedule(static)
      for (int i = 0; i < n; ++i) {
        double *ui = &u[((size_t)t * n + i) * H];
        matvec(v.C1[t], v.c1[t], &m[(size_t)i * H], H, H, ui);
        for (int c = 0; c < H; ++c) tmp[c] = silu(ui[c]);
        matvec(v.C2[t], v.c2[t], tmp, H, H, &hn[(size_t)i * H]);
        for (int c = 0; c < H; ++c) hn[(size_t)i * H + c] += hp[(size_t)i * H + c];
      }
      free(tmp);
    }
  }
  /* readout: per-atom energies side by side, then their sum in atom order */
  double E = 0.0;
  const double *hT = &h[(size_t)T * n * H];
  double *ea = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
#pragma omp parallel
  {
    double *y = (double *)malloc(sizeof(double) * RH);
#pragma omp for schedule(static)
    for (int i = 0; i < n; ++i) {
      matvec(v.W1, v.b1, &hT[(size_t)i * H], RH, H, y);
      double ei = v.b2[0];
      for (int o = 0; o < RH; ++o) ei += v.w2[o] * silu(y[o]);
      ea[i] = ei;
    }
    free(y);
  }
  for (int i = 0; i < n; ++i) E += ea[i];
  E *= M->scale;
  free(ea);

  if (F) {
    /* backward: gh = dE/dh^t, per atom */
    double *gh = (double *)calloc((size_t)n * H, sizeof(double));
    double *gp = (double *)calloc((size_t)n * H, sizeof(double));
    double *gm = (double *)malloc(sizeof(double) * (size_t)n * H);
    double *gx = (double *)malloc(sizeof(double) * (size_t)n * H);
    double *gr = (double *)calloc((size_t)(np > 0 ? np : 1), sizeof(double));
#pragma omp parallel
    {
      double *y = (double *)malloc(sizeof(double) * RH);
      double *g = (double *)malloc(sizeof(double) * RH);
#pragma omp for schedule(static)
      for (int i = 0; i < n; ++i) {
        matvec(v.W1, v.b1, &hT[(size_t)i * H], RH, H, y);
        for (int o = 0; o < RH; ++o) g[o] = M->scale * v.w2[o] * dsilu(y[o]);
        matvec_t_acc(v.W1, g, RH, H, &gh[(size_t)i * H]);
      }
      free(y); free(g);
    }
    for (int t = T - 1; t >= 0; --t) {
      const double *xt = &xb[(size_t)t * n * H];
      /* through h^{t+1} = h^t + C2 silu(u) + c2 and u = C1 m + c1 */
      memcpy(gp, gh, sizeof(double) * (size_t)n * H); /* residual */
      memset(gm, 0, sizeof(double) * (size_t)n * H);
#pragma omp parallel
      {
        double *gs = (double *)malloc(sizeof(double) * H);
#pragma omp for schedule(static)
        for (int i = 0; i < n; ++i) {
          const double *ui = &u[((size_t)t * n + i) * H];
          memset(gs, 0, sizeof(double) * H);
          matvec_t_acc(v.C2[t], &gh[(size_t)i * H], H, H, gs);
          for (int c = 0; c < H; ++c) gs[c] *= dsilu(ui[c]);
          matvec_t_acc(v.C1[t], gs, H, H, &gm[(size_t)i * H]);
        }
        free(gs);
      }
      /* through m_i = sum_j W_ij (.) x_j */
      memset(gx, 0, sizeof(double) * (size_t)n * H);
      for (long k0 = 0; k0 < np; k0 += chunk) {
        long k1 = k0 + chunk < np ? k0 + chunk : np;
        filter_chunk(M, &v, t, k0, k1, e, de, fc, dfc, Wc, dWc);
        for (long k = k0; k < k1; ++k) {
          int i = P[5 * k], j = P[5 * k + 1];
          const double *Wf = &Wc[(size_t)(k - k0) * H], *dWf = &dWc[(size_t)(k - k0) * H];
          double s = 0.0;
          for (int c = 0; c < H; ++c) {
            double gw = gm[(size_t)i * H + c] * xt[(size_t)j * H + c];
            s += gw * dWf[c];
            gx[(size_t)j * H + c] += Wf[c] * gm[(size_t)i * H + c];
          }
          gr[k] += s;
        }
      }
      /* through x_j = B h_j */
#pragma omp parallel for schedule(static)
      for (int j = 0; j < n; ++j) matvec_t_acc(v.B[t], &gx[(size_t)j * H], H, H, &gp[(size_t)j * H]);
      memcpy(gh, gp, sizeof(double) * (size_t)n * H);
    }
    /* F = -dE/dq; r_ij depends on q_i and q_j: dr/dq_j = d/r, dr/dq_i = -d/r */
    memset(F, 0, sizeof(double) * 3 * (size_t)n);
    for (long k = 0; k < np; ++k) {
      int i = P[5 * k], j = P[5 * k + 1];
      for (int a = 0; a < 3; ++a) {
        double dq = gr[k] * d[3 * k + a] / r[k];
        F[3 * i + a] += dq;
        F[3 * j + a] -= dq;
      }
    }
    free(gh); free(gp); free(gm); free(gx); free(gr);
  }
  free(P); free(d); free(r); free(e); free(de); free(fc); free(dfc);
  free(h); free(xb); free(u); free(m); free(Wc); free(dWc);
  return E;
}

/* The network as a force field of the integrator and window code
 * (lsd_oracle.c, kind ORA_POT_EXT): context = the network and the species of
 * the atoms. */
typedef struct {
  const ora_mpnn *m;
  const int32_t *species;
} ora_mpnn_ctx;

double ora_mpnn_ext(const void *ctx, int n, const double *x, double L, double *F) {
  const ora_mpnn_ctx *c = (const ora_mpnn_ctx *)ctx;
  return ora_mpnn_energy_forces(c->m, n, c->species, x, L, F);
}
