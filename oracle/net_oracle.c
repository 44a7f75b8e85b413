/*
 * net_oracle.c -- plain FP64 learned many-body draft: forces, the gradient
 * of the force-matching loss, and the Adam update.
 *
 * TEST INFRASTRUCTURE ONLY (see lsd_oracle.c).  The paper's drafts are small
 * machine-learned potentials trained to reproduce the target's forces, and
 * they predict forces directly rather than as energy gradients; LSD accepts a
 * non-conservative draft because its samples are corrected by verification
 * (Sec. 3, Sec. 4).  The draft defined here is a one-layer direct-force
 * network over a species-resolved radial descriptor (H = 32 hidden units,
 * S species, B radial functions, cutoff rc):
 *
 *   pairs     (i, j, n) with d = q_j + n L - q_i, r = |d| < rc
 *   e_b(r)  = f_c(r) sin(b pi r / rc) / r,  b = 1..B,
 *             f_c(r) = (cos(pi r / rc) + 1) / 2
 *   D_i     = sum over pairs (i, j, n) of e(r) in the block of species s_j
 *             (S B entries: D_i[s B + b-1])
 *   z_i     = W1 D_i + b1[s_i],  h_i = silu(z_i) = z / (1 + exp(-z))
 *   v_i     = W2 h_i  (B entries)
 *   f_ij    = sum_b e_b(r) (c[t(s_i, s_j)][b] + v_i[b] + v_j[b])
 *   F_i     = - sum over pairs (i, j, n) of f_ij d / r
 *
 * f_ij is symmetric in i and j, so the forces obey Newton's third law; with
 * v = 0 the draft is the pair draft of pair_oracle.c with weights c.
 * Parameters, one flat vector, matrices stored [out][in]:
 *   W1 [H][S B], b1 [S][H], W2 [B][H], c [S(S+1)/2][B].
 *
 * Force matching minimises the squared error of all force components against
 * reference forces Y; ora_net_sse_grad returns sum |F - Y|^2 over one frame
 * and adds its gradient in the parameters, by the chain rule through the
 * forward pass above, term by term (ora_net_backward: the same chain rule
 * for any loss whose derivative in the forces is given).  ora_net_adam is
 * one step of Adam (Kingma and Ba, 2015) with bias-corrected moments.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NET_H 32

long ora_pairs_brute(int n, const double *x, double L, double rc, int32_t *out, long cap);
long ora_pairs_cells(int n, const double *x, double L, double rc, int32_t *out, long cap);
int ora_pair_types(int S);
int ora_pair_type(int a, int b, int S);

int ora_net_param_count(int S, int B) {
  return NET_H * S * B + S * NET_H + B * NET_H + ora_pair_types(S) * B;
}

static long records(int n, const double *x, double L, double rc, int32_t **out) {
  int cells = floor(L / rc) >= 3;
  long np = cells ? ora_pairs_cells(n, x, L, rc, NULL, 0) : ora_pairs_brute(n, x, L, rc, NULL, 0);
  *out = (int32_t *)malloc(sizeof(int32_t) * 5 * (size_t)(np > 0 ? np : 1));
  if (cells) ora_pairs_cells(n, x, L, rc, *out, np);
  else ora_pairs_brute(n, x, L, rc, *out, np);
  return np;
}

static void geometry(const double *x, double L, const int32_t *rec, double d[3], double *r) {
  int i = rec[0], j = rec[1];
  for (int a = 0; a < 3; ++a) d[a] = (x[3 * j + a] - x[3 * i + a]) + (double)rec[2 + a] * L;
  *r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
}

static void radial(double r, double rc, int B, double *e) {
  const double pi = 3.14159265358979323846;
  double fc = 0.5 * (cos(pi * r / rc) + 1.0);
  for (int b = 1; b <= B; ++b) e[b - 1] = fc * sin(b * pi * r / rc) / r;
}

static double sigmoid(double z) { return 1.0 / (1.0 + exp(-z)); }

typedef struct {
  const double *W1, *b1, *W2, *c;
} Params;

static Params unpack(const double *p, int S, int B) {
  Params q;
  q.W1 = p;
  q.b1 = q.W1 + NET_H * S * B;
  q.W2 = q.b1 + S * NET_H;
  q.c = q.W2 + B * NET_H;
  return q;
}

/* descriptor, pre-activation and edge coefficients of every atom */
static void nodes(int n, const double *x, double L, const int32_t *sp, int S, int B, double rc,
                  Params w, const int32_t *rec, long np, double *D, double *z, double *v) {
  const int Din = S * B;
  double e[64];
  memset(D, 0, sizeof(double) * (size_t)n * Din);
  for (long p = 0; p < np; ++p) {
    const int32_t *q = &rec[5 * p];
    double d[3], r;
    geometry(x, L, q, d, &r);
    radial(r, rc, B, e);
    for (int b = 0; b < B; ++b) D[(size_t)q[0] * Din + sp[q[1]] * B + b] += e[b];
  }
  for (int i = 0; i < n; ++i) {
    double hh[NET_H];
    for (int h = 0; h < NET_H; ++h) {
      double s = w.b1[sp[i] * NET_H + h];
      for (int k = 0; k < Din; ++k) s += w.W1[h * Din + k] * D[(size_t)i * Din + k];
      z[(size_t)i * NET_H + h] = s;
      hh[h] = s * sigmoid(s);
    }
    for (int b = 0; b < B; ++b) {
      double s = 0.0;
      for (int h = 0; h < NET_H; ++h) s += w.W2[b * NET_H + h] * hh[h];
      v[(size_t)i * B + b] = s;
    }
  }
}

/* F[n][3]; D [n][S B], z [n][H], v [n][B] are returned when non-NULL */
void ora_net_forward(int n, const double *x, double L, const int32_t *sp, int S, int B, double rc,
                     const double *params, double *D_out, double *z_out, double *v_out,
                     double *F) {
  Params w = unpack(params, S, B);
  int32_t *rec;
  long np = records(n, x, L, rc, &rec);
  double *D = (double *)malloc(sizeof(double) * (size_t)n * S * B + 8);
  double *z = (double *)malloc(sizeof(double) * (size_t)n * NET_H + 8);
  double *v = (double *)malloc(sizeof(double) * (size_t)n * B + 8);
  nodes(n, x, L, sp, S, B, rc, w, rec, np, D, z, v);
  double e[64];
  memset(F, 0, sizeof(double) * 3 * (size_t)n);
  for (long p = 0; p < np; ++p) {
    const int32_t *q = &rec[5 * p];
    double d[3], r;
    geometry(x, L, q, d, &r);
    radial(r, rc, B, e);
    const double *ct = w.c + (size_t)ora_pair_type(sp[q[0]], sp[q[1]], S) * B;
    double f = 0.0;
    for (int b = 0; b < B; ++b) f += e[b] * (ct[b] + v[(size_t)q[0] * B + b] + v[(size_t)q[1] * B + b]);
    for (int a = 0; a < 3; ++a) F[3 * q[0] + a] -= f * d[a] / r;
  }
  if (D_out) memcpy(D_out, D, sizeof(double) * (size_t)n * S * B);
  if (z_out) memcpy(z_out, z, sizeof(double) * (size_t)n * NET_H);
  if (v_out) memcpy(v_out, v, sizeof(double) * (size_t)n * B);
  free(D);
  free(z);
  free(v);
  free(rec);
}

/* adds sum_i G_i . dF_i/dtheta to grad[P] (G [n][3] = dLoss/dF) */
static void backprop(int n, const double *x, double L, const int32_t *sp, int S, int B, double rc,
                     Params w, const int32_t *rec, long np, const double *D, const double *z,
                     const double *G, double *grad) {
  const int Din = S * B;
  double *gW1 = grad, *gb1 = gW1 + NET_H * Din, *gW2 = gb1 + S * NET_H, *gc = gW2 + B * NET_H;
  double *dv = (double *)calloc((size_t)n * B + 1, sizeof(double));
  double e[64];
  /* each pair term -f d / r of F_i: dLoss/df = -G_i . d / r, and f depends
   * on c[t], v_i and v_j with coefficient e_b */
  for (long p = 0; p < np; ++p) {
    const int32_t *q = &rec[5 * p];
    double d[3], r;
    geometry(x, L, q, d, &r);
    radial(r, rc, B, e);
    double df = 0.0;
    for (int a = 0; a < 3; ++a) df -= G[3 * q[0] + a] * d[a] / r;
    const int t = ora_pair_type(sp[q[0]], sp[q[1]], S);
    for (int b = 0; b < B; ++b) {
      gc[(size_t)t * B + b] += df * e[b];
      dv[(size_t)q[0] * B + b] += df * e[b];
      dv[(size_t)q[1] * B + b] += df * e[b];
    }
  }
  /* v_i = W2 h_i, h_i = silu(z_i), z_i = W1 D_i + b1[s_i] */
  for (int i = 0; i < n; ++i) {
    const double *zi = z + (size_t)i * NET_H;
    const double *dvi = dv + (size_t)i * B;
    for (int h = 0; h < NET_H; ++h) {
      double sg = sigmoid(zi[h]);
      double hh = zi[h] * sg;
      double dh = 0.0;
      for (int b = 0; b < B; ++b) {
        gW2[b * NET_H + h] += dvi[b] * hh;
        dh += w.W2[b * NET_H + h] * dvi[b];
      }
      double dz = dh * (sg * (1.0 + zi[h] * (1.0 - sg)));
      gb1[sp[i] * NET_H + h] += dz;
      for (int k = 0; k < Din; ++k) gW1[h * Din + k] += dz * D[(size_t)i * Din + k];
    }
  }
  free(dv);
}

/* adds sum_i G_i . dF_i/dtheta (G [n][3]) to grad[P]: the gradient of any
 * loss of the forces whose derivative in F is G */
void ora_net_backward(int n, const double *x, double L, const int32_t *sp, int S, int B, double rc,
                      const double *params, const double *G, double *grad) {
  Params w = unpack(params, S, B);
  int32_t *rec;
  long np = records(n, x, L, rc, &rec);
  double *D = (double *)malloc(sizeof(double) * (size_t)n * S * B + 8);
  double *z = (double *)malloc(sizeof(double) * (size_t)n * NET_H + 8);
  double *v = (double *)malloc(sizeof(double) * (size_t)n * B + 8);
  nodes(n, x, L, sp, S, B, rc, w, rec, np, D, z, v);
  backprop(n, x, L, sp, S, B, rc, w, rec, np, D, z, G, grad);
  free(D);
  free(z);
  free(v);
  free(rec);
}

/* returns sum_i |F_i - Y_i|^2 and adds its gradient to grad[P] */
double ora_net_sse_grad(int n, const double *x, double L, const int32_t *sp, int S, int B,
                        double rc, const double *params, const double *Y, double *grad) {
  double *F = (double *)malloc(sizeof(double) * (3 * (size_t)n + 1));
  double *G = (double *)malloc(sizeof(double) * (3 * (size_t)n + 1));
  ora_net_forward(n, x, L, sp, S, B, rc, params, NULL, NULL, NULL, F);
  double sse = 0.0;
  for (size_t k = 0; k < 3 * (size_t)n; ++k) {
    double res = F[k] - Y[k];
    sse += res * res;
    G[k] = 2.0 * res;
  }
  ora_net_backward(n, x, L, sp, S, B, rc, params, G, grad);
  free(F);
  free(G);
  return sse;
}

/* one Adam step at step count t >= 1 on P parameters with gradient g */
void ora_net_adam(int P, double *params, double *m, double *v, const double *g, double lr,
                  double beta1, double beta2, double eps, long t) {
  const double c1 = 1.0 - pow(beta1, (double)t), c2 = 1.0 - pow(beta2, (double)t);
  for (int k = 0; k < P; ++k) {
    m[k] = beta1 * m[k] + (1.0 - beta1) * g[k];
    v[k] = beta2 * v[k] + (1.0 - beta2) * g[k] * g[k];
    double mh = m[k] / c1, vh = v[k] / c2;
    params[k] -= lr * mh / (sqrt(vh) + eps);
  }
}

/* The learned draft as a force field of the integrator and window code
 * (lsd_oracle.c, kind ORA_POT_EXT).  A direct-force draft has no energy; 0
 * is returned. */
typedef struct {
  int S, B;
  double rc;
  const double *params;
  const int32_t *species;
} ora_net_ctx;

double ora_net_ext(const void *ctx, int n, const double *x, double L, double *F) {
  const ora_net_ctx *c = (const ora_net_ctx *)ctx;
  ora_net_forward(n, x, L, c->species, c->S, c->B, c->rc, c->params, NULL, NULL, NULL, F);
  return 0.0;
}
