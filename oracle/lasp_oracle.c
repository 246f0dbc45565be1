/*
 * FP64 CPU oracle for grouped full-spectrum fitting (LASP-Adam-GPU).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant generator with the HIP library; physical
 * constants and the feature table are written out here on purpose.
 *
 * For one spectrum at a time, in double precision throughout (FP32 inputs are
 * promoted exactly), it evaluates the model of Section 2.2 in the paper's
 * order and notation:
 *
 *   Eq. 1   model spectrum from the interpolator: F'_c = sum_k phi_k(x) B_k,c
 *   Eq. 5   Gaussian kernel G(mu, sigma) of 2*ceil(|mu|+5 sigma)+1 taps and
 *           the convolution F'' = F' (x) G
 *   Eq. 6   multiplicative continuum (P(x) b)^T (.) F'' with Legendre
 *           polynomials of degree 0..D at x_j = -1 + 2 (j-1)/p, b by weighted
 *           least squares (direct Gram matrix, Cholesky)
 *   Eq. 7   residual eps = o - C (.) F''
 *   Eq. 9   objective, read per spectrum as chi2 / n_eff with W = ivar
 *
 * and fits it with a textbook Levenberg-Marquardt iteration (Marquardt 1963;
 * the damped Gauss-Newton method of Nocedal & Wright, ch. 10), which reaches
 * the same minimiser that the paper's curve_fit path and Adam path target.
 * The covariance follows the linear error propagation of the "Estimating
 * parameter errors" stage.  Readings of points the paper leaves open:
 *   - kernel in pixels, mu > 0 is a redshift, unit-sum discrete Gaussian over
 *     exactly m = -H..H, H = min(ceil(|mu| + 5 sigma), M);
 *   - mu = RV / (c ln10 dlog10), sigma_px = max(sigma / (c ln10 dlog10), 0.1);
 *   - per-arm instrument term sigma_eff = sqrt(sigma^2 + sigma_arm^2);
 *   - the basis spans the pixel range plus M margin columns on each side,
 *     so no edge pixel is excluded;
 *   - free parameters normalised to [-1, 1] over a fixed box, no clamping;
 *   - pixels with non-finite data or ivar <= 0 get weight zero.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_NB 20          /* interpolator terms */
#define ORC_NP 5           /* free parameters per spectrum */
#define ORC_DMAX 24        /* largest continuum degree accepted */
#define ORC_CKMS 299792.458
#define ORC_LN10 2.302585092994045684
#define ORC_SIGMA_FLOOR 0.1

enum {
  ORC_NONFINITE = 1u << 0,
  ORC_NO_DATA = 1u << 1,
  ORC_SINGULAR = 1u << 2,
  ORC_CONT_NONPOS = 1u << 3,
  ORC_OUT_OF_BOX = 1u << 4,
  ORC_NOT_CONVERGED = 1u << 5,
  ORC_WIDTH_FLOOR = 1u << 6, /* kernel width at the 0.1 px floor in some arm */
};

typedef struct orc_cfg {
  int n_pix;          /* p */
  int margin;         /* M: basis has n_pix + 2M columns, column c <-> pixel c - M */
  int degree;         /* D */
  int n_arms;         /* 0: one arm without instrument term */
  int arm_start[4];
  double arm_sigma[4];
  double dlog10;      /* grid step in log10(lambda) */
  double lo[ORC_NP], hi[ORC_NP];
  int n_classes;      /* 1, or 3 (cool, warm, hot emulator classes) */
  double edges[4];    /* Teff regime edges (K) of the 3-class emulator */
} orc_cfg;

/* Exponents of x1, x2, x3 for each interpolator term: total degree <= 3,
 * graded, lexicographic within a degree. */
static const int ORC_EXP[ORC_NB][3] = {
    {0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {2, 0, 0}, {1, 1, 0}, {1, 0, 1},
    {0, 2, 0}, {0, 1, 1}, {0, 0, 2}, {3, 0, 0}, {2, 1, 0}, {2, 0, 1}, {1, 2, 0},
    {1, 1, 1}, {1, 0, 2}, {0, 3, 0}, {0, 2, 1}, {0, 1, 2}, {0, 0, 3}};

static double ipow(double x, int e) {
  double r = 1.0;
  for (int i = 0; i < e; ++i) r *= x;
  return r;
}

/* Eq. 1: phi_k(x) and d phi_k / d x_t (dphi[t*20 + k]). */
void orc_features(const double *x, double *phi, double *dphi) {
  for (int k = 0; k < ORC_NB; ++k) {
    const int *e = ORC_EXP[k];
    phi[k] = ipow(x[0], e[0]) * ipow(x[1], e[1]) * ipow(x[2], e[2]);
    if (dphi) {
      for (int t = 0; t < 3; ++t) {
        double d = 0.0;
        if (e[t] > 0) {
          d = e[t];
          for (int s = 0; s < 3; ++s) d *= ipow(x[s], s == t ? e[s] - 1 : e[s]);
        }
        dphi[t * ORC_NB + k] = d;
      }
    }
  }
}

/* Legendre polynomial P_n(x) by the three-term recurrence
 * (n+1) P_{n+1} = (2n+1) x P_n - n P_{n-1}. */
double orc_legendre(int n, double x) {
  if (n == 0) return 1.0;
  double pm = 1.0, p = x;
  for (int k = 1; k < n; ++k) {
    double pn = ((2.0 * k + 1.0) * x * p - k * pm) / (k + 1.0);
    pm = p;
    p = pn;
  }
  return p;
}

/* Node of pixel j (0-based): x = -1 + 2 j / p, the paper's x_j with j-1. */
static double orc_node(int j, int p) { return -1.0 + 2.0 * (double)j / (double)p; }

/* Eq. 5 kernel.  mu, sig in pixels (sig already floored).  Writes G[m+H],
 * dG/dmu and dG/dsig for m = -H..H and returns H. */
int orc_kernel(double mu, double sig, int margin, double *G, double *dGdmu, double *dGdsig) {
  int H = (int)ceil(fabs(mu) + 5.0 * sig);
  if (H > margin) H = margin;
  double sum = 0.0, s1 = 0.0, s2 = 0.0;
  for (int m = -H; m <= H; ++m) {
    double d = m - mu;
    double g = exp(-d * d / (2.0 * sig * sig));
    G[m + H] = g;
    sum += g;
  }
  for (int m = -H; m <= H; ++m) {
    double d = m - mu;
    G[m + H] /= sum;
    s1 += G[m + H] * d;
    s2 += G[m + H] * d * d;
  }
  for (int m = -H; m <= H; ++m) {
    double d = m - mu;
    double gm = G[m + H];
    if (dGdmu) dGdmu[m + H] = gm * (d - s1) / (sig * sig);
    if (dGdsig) dGdsig[m + H] = gm * (d * d - s2) / (sig * sig * sig);
  }
  return H;
}

/* F''_j = sum_{m=-H..H} G[m] F'[j - m + M] (indices clamped to the basis
 * range; with H <= M the clamp never triggers). */
void orc_convolve(const double *fp, int n_ext, const double *G, int H, int margin, int j0, int j1,
                  double *out) {
  for (int j = j0; j < j1; ++j) {
    double acc = 0.0;
    for (int m = -H; m <= H; ++m) {
      int c = j - m + margin;
      if (c < 0) c = 0;
      if (c > n_ext - 1) c = n_ext - 1;
      acc += G[m + H] * fp[c];
    }
    out[j] = acc;
  }
}

/* Decoded parameters and the pixel-unit kernel quantities of one arm. */
typedef struct {
  double mu, sig;          /* pixels */
  double dmu_du, dsig_du;  /* d mu / d u4, d sig / d u5 (0 when floored) */
  int floored;             /* the width sits at the 0.1 px floor */
} orc_arm_kernel;

static void arm_kernel(const orc_cfg *cfg, const double *u, int arm, orc_arm_kernel *ak) {
  const double scale = ORC_CKMS * ORC_LN10 * cfg->dlog10; /* km/s per pixel */
  double rv = cfg->lo[3] + 0.5 * (u[3] + 1.0) * (cfg->hi[3] - cfg->lo[3]);
  double sg = cfg->lo[4] + 0.5 * (u[4] + 1.0) * (cfg->hi[4] - cfg->lo[4]);
  double sinst = (cfg->n_arms > 0) ? cfg->arm_sigma[arm] : 0.0;
  double seff = (cfg->n_arms > 0) ? sqrt(sg * sg + sinst * sinst) : sg;
  double dseff = (cfg->n_arms > 0) ? (seff > 0.0 ? sg / seff : 0.0) : 1.0;
  ak->mu = rv / scale;
  ak->dmu_du = 0.5 * (cfg->hi[3] - cfg->lo[3]) / scale;
  double spx = seff / scale;
  if (spx < ORC_SIGMA_FLOOR) {
    ak->sig = ORC_SIGMA_FLOOR;
    ak->dsig_du = 0.0;
    ak->floored = 1;
  } else {
    ak->sig = spx;
    ak->dsig_du = 0.5 * (cfg->hi[4] - cfg->lo[4]) * dseff / scale;
    ak->floored = 0;
  }
}

static int arm_count(const orc_cfg *cfg) { return cfg->n_arms > 0 ? cfg->n_arms : 1; }

/* ORC_WIDTH_FLOOR if the width of some arm is floored at u. */
static unsigned floor_flag(const orc_cfg *cfg, const double *u) {
  for (int a = 0; a < arm_count(cfg); ++a) {
    orc_arm_kernel ak;
    arm_kernel(cfg, u, a, &ak);
    if (ak.floored) return ORC_WIDTH_FLOOR;
  }
  return 0;
}
static int arm_begin(const orc_cfg *cfg, int a) { return cfg->n_arms > 0 ? cfg->arm_start[a] : 0; }
static int arm_end(const orc_cfg *cfg, int a) {
  return (cfg->n_arms > 0 && a + 1 < cfg->n_arms) ? cfg->arm_start[a + 1] : cfg->n_pix;
}

/* Cholesky factorisation of a symmetric n x n matrix (row-major, in place,
 * lower triangle).  Returns 0 on success, -1 if not positive definite. */
static int chol(double *a, int n) {
  for (int j = 0; j < n; ++j) {
    double d = a[j * n + j];
    for (int k = 0; k < j; ++k) d -= a[j * n + k] * a[j * n + k];
    if (!(d > 0.0) || !isfinite(d)) return -1;
    d = sqrt(d);
    a[j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double s = a[i * n + j];
      for (int k = 0; k < j; ++k) s -= a[i * n + k] * a[j * n + k];
      a[i * n + j] = s / d;
    }
  }
  return 0;
}

static void chol_solve(const double *l, int n, double *x) {
  for (int i = 0; i < n; ++i) {
    double s = x[i];
    for (int k = 0; k < i; ++k) s -= l[i * n + k] * x[k];
    x[i] = s / l[i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = x[i];
    for (int k = i + 1; k < n; ++k) s -= l[k * n + i] * x[k];
    x[i] = s / l[i * n + i];
  }
}

/* Inverse of an SPD matrix from its Cholesky factor (column by column). */
static void chol_inverse(const double *l, int n, double *inv) {
  double *e = (double *)malloc(sizeof(double) * n);
  for (int c = 0; c < n; ++c) {
    for (int i = 0; i < n; ++i) e[i] = (i == c) ? 1.0 : 0.0;
    chol_solve(l, n, e);
    for (int i = 0; i < n; ++i) inv[i * n + c] = e[i];
  }
  free(e);
}

/* Everything the model produces at fixed normalised parameters u. */
typedef struct {
  double *fp;     /* [n_ext]  F' */
  double *fpp;    /* [P]      F'' */
  double *dfpp;   /* [5][P]   d F'' / d u_t */
  double *w;      /* [P]      weights */
  double *o;      /* [P]      data (0 where w = 0) */
  double *leg;    /* [P][D+1] Legendre design */
  int n_eff;
  unsigned flags;
} orc_work;

static void work_alloc(const orc_cfg *cfg, orc_work *wk) {
  int P = cfg->n_pix, ne = P + 2 * cfg->margin, nd = cfg->degree + 1;
  wk->fp = (double *)calloc(ne, sizeof(double));
  wk->fpp = (double *)calloc(P, sizeof(double));
  wk->dfpp = (double *)calloc((size_t)ORC_NP * P, sizeof(double));
  wk->w = (double *)calloc(P, sizeof(double));
  wk->o = (double *)calloc(P, sizeof(double));
  wk->leg = (double *)calloc((size_t)P * nd, sizeof(double));
}

static void work_free(orc_work *wk) {
  free(wk->fp);
  free(wk->fpp);
  free(wk->dfpp);
  free(wk->w);
  free(wk->o);
  free(wk->leg);
}

/* Weights, data and Legendre design: fixed for the whole fit. */
static void setup_data(const orc_cfg *cfg, const float *obs, const float *ivar, orc_work *wk) {
  int P = cfg->n_pix, nd = cfg->degree + 1;
  wk->n_eff = 0;
  wk->flags = 0;
  for (int j = 0; j < P; ++j) {
    double o = obs[j], iv = ivar[j];
    if (!isfinite(o) || !isfinite(iv)) wk->flags |= ORC_NONFINITE;
    if (isfinite(o) && isfinite(iv) && iv > 0.0) {
      wk->w[j] = iv;
      wk->o[j] = o;
      wk->n_eff++;
    } else {
      wk->w[j] = 0.0;
      wk->o[j] = 0.0;
    }
    double x = orc_node(j, P);
    for (int n = 0; n < nd; ++n) wk->leg[(size_t)j * nd + n] = orc_legendre(n, x);
  }
}

/*
 * Weights of the emulator's temperature classes (Eq. 1 with the five Teff
 * regimes of the ELODIE emulator): with a = clamp((T - e0) / (e1 - e0)) and
 * b = clamp((T - e2) / (e3 - e2)), the cool, warm and hot classes weigh
 * 1 - a, a (1 - b) and a b -- one class inside a regime, a linear blend in
 * Teff across the two transition regimes.  dw[] is d w / d u_1 (zero where
 * the blend is flat).  One class: w = 1.
 */
void orc_class_weights(const orc_cfg *cfg, const double *u, double *w, double *dw) {
  if (cfg->n_classes <= 1) {
    w[0] = 1.0;
    dw[0] = 0.0;
    return;
  }
  const double lt = cfg->lo[0] + 0.5 * (u[0] + 1.0) * (cfg->hi[0] - cfg->lo[0]);
  const double T = pow(10.0, lt);
  const double dT = T * ORC_LN10 * 0.5 * (cfg->hi[0] - cfg->lo[0]);
  const double *e = cfg->edges;
  double a = (T - e[0]) / (e[1] - e[0]), da = dT / (e[1] - e[0]);
  if (!(T > e[0] && T < e[1])) da = 0.0;
  a = a < 0.0 ? 0.0 : (a > 1.0 ? 1.0 : a);
  double b = (T - e[2]) / (e[3] - e[2]), db = dT / (e[3] - e[2]);
  if (!(T > e[2] && T < e[3])) db = 0.0;
  b = b < 0.0 ? 0.0 : (b > 1.0 ? 1.0 : b);
  w[0] = 1.0 - a;
  w[1] = a * (1.0 - b);
  w[2] = a * b;
  dw[0] = -da;
  dw[1] = da * (1.0 - b) - a * db;
  dw[2] = da * b + a * db;
}

/* Eq. 1 and Eq. 5 with derivatives: F', F'' and dF''/du at u. */
static void model_spectrum(const orc_cfg *cfg, const float *basis, const double *u, orc_work *wk,
                           int want_deriv) {
  int P = cfg->n_pix, M = cfg->margin, ne = P + 2 * M;
  const int ncl = cfg->n_classes > 1 ? cfg->n_classes : 1;
  double phi[ORC_NB], dphi[3 * ORC_NB], cw[3], dcw[3];
  orc_features(u, phi, dphi);
  orc_class_weights(cfg, u, cw, dcw);
  double *dfp = (double *)calloc((size_t)3 * ne, sizeof(double));
  for (int c = 0; c < ne; ++c) {
    double acc = 0.0, d0 = 0.0, d1 = 0.0, d2 = 0.0;
    for (int q = 0; q < ncl; ++q)
      for (int k = 0; k < ORC_NB; ++k) {
        double b = basis[((size_t)q * ORC_NB + k) * ne + c];
        acc += cw[q] * phi[k] * b;
        d0 += (dcw[q] * phi[k] + cw[q] * dphi[k]) * b;
        d1 += cw[q] * dphi[ORC_NB + k] * b;
        d2 += cw[q] * dphi[2 * ORC_NB + k] * b;
      }
    wk->fp[c] = acc;
    dfp[c] = d0;
    dfp[ne + c] = d1;
    dfp[2 * ne + c] = d2;
  }
  int Gmax = 2 * M + 1;
  double *G = (double *)malloc(sizeof(double) * Gmax);
  double *Gm = (double *)malloc(sizeof(double) * Gmax);
  double *Gs = (double *)malloc(sizeof(double) * Gmax);
  for (int a = 0; a < arm_count(cfg); ++a) {
    orc_arm_kernel ak;
    arm_kernel(cfg, u, a, &ak);
    int H = orc_kernel(ak.mu, ak.sig, M, G, Gm, Gs);
    int j0 = arm_begin(cfg, a), j1 = arm_end(cfg, a);
    orc_convolve(wk->fp, ne, G, H, M, j0, j1, wk->fpp);
    if (want_deriv) {
      for (int t = 0; t < 3; ++t)
        orc_convolve(dfp + (size_t)t * ne, ne, G, H, M, j0, j1, wk->dfpp + (size_t)t * P);
      orc_convolve(wk->fp, ne, Gm, H, M, j0, j1, wk->dfpp + (size_t)3 * P);
      orc_convolve(wk->fp, ne, Gs, H, M, j0, j1, wk->dfpp + (size_t)4 * P);
      for (int j = j0; j < j1; ++j) {
        wk->dfpp[(size_t)3 * P + j] *= ak.dmu_du;
        wk->dfpp[(size_t)4 * P + j] *= ak.dsig_du;
      }
    }
  }
  free(G);
  free(Gm);
  free(Gs);
  free(dfp);
}

/* Eq. 6: weighted least squares for the Legendre coefficients b. */
static int continuum_ls(const orc_cfg *cfg, const orc_work *wk, double *b) {
  int P = cfg->n_pix, nd = cfg->degree + 1;
  double A[(ORC_DMAX + 1) * (ORC_DMAX + 1)];
  memset(A, 0, sizeof(double) * nd * nd);
  for (int n = 0; n < nd; ++n) b[n] = 0.0;
  for (int j = 0; j < P; ++j) {
    double wf = wk->w[j] * wk->fpp[j];
    const double *L = wk->leg + (size_t)j * nd;
    for (int m = 0; m < nd; ++m) {
      b[m] += wf * wk->o[j] * L[m];
      for (int n = 0; n <= m; ++n) A[m * nd + n] += wf * wk->fpp[j] * L[m] * L[n];
    }
  }
  for (int m = 0; m < nd; ++m)
    for (int n = m + 1; n < nd; ++n) A[m * nd + n] = A[n * nd + m];
  if (chol(A, nd) != 0) return -1;
  chol_solve(A, nd, b);
  return 0;
}

static double cont_at(const orc_cfg *cfg, const orc_work *wk, const double *b, int j) {
  int nd = cfg->degree + 1;
  double c = 0.0;
  for (int n = 0; n < nd; ++n) c += b[n] * wk->leg[(size_t)j * nd + n];
  return c;
}

/* Eqs. 7 and 9: chi2 = sum W (o - C F'')^2 at coefficients b. */
static double chi2_at(const orc_cfg *cfg, const orc_work *wk, const double *b) {
  double s = 0.0;
  for (int j = 0; j < cfg->n_pix; ++j) {
    double e = wk->o[j] - cont_at(cfg, wk, b, j) * wk->fpp[j];
    s += wk->w[j] * e * e;
  }
  return s;
}

/*
 * Model at fixed normalised parameters u (5 values).  Outputs, each optional:
 *   fp[n_ext] F', fpp[P] F'', b[D+1] Legendre coefficients, model[P] = C F'',
 *   chi2, n_eff, grad[5] = d(chi2/n_eff)/du with b at its least-squares value
 *   (envelope theorem), jac[5][P] = d model / d u at fixed b, flags.
 * Returns 0, or -1 if the normal equations are not positive definite.
 */
int orc_eval(const orc_cfg *cfg, const float *obs, const float *ivar, const float *basis,
             const double *u, double *fp, double *fpp, double *b_out, double *model, double *chi2,
             int *n_eff, double *grad, double *jac, unsigned *flags) {
  int P = cfg->n_pix, ne = P + 2 * cfg->margin, nd = cfg->degree + 1;
  if (nd > ORC_DMAX + 1) return -2;
  orc_work wk;
  work_alloc(cfg, &wk);
  setup_data(cfg, obs, ivar, &wk);
  model_spectrum(cfg, basis, u, &wk, grad != NULL || jac != NULL);
  double b[ORC_DMAX + 1];
  int rc = 0;
  unsigned fl = wk.flags;
  if (wk.n_eff <= ORC_NP + nd) fl |= ORC_NO_DATA;
  if (continuum_ls(cfg, &wk, b) != 0) {
    fl |= ORC_SINGULAR;
    rc = -1;
    for (int n = 0; n < nd; ++n) b[n] = NAN;
  }
  double g[ORC_NP] = {0, 0, 0, 0, 0};
  double s = 0.0;
  for (int j = 0; j < P; ++j) {
    double c = cont_at(cfg, &wk, b, j);
    if (!(c > 0.0)) fl |= ORC_CONT_NONPOS;
    double m = c * wk.fpp[j];
    double e = wk.o[j] - m;
    s += wk.w[j] * e * e;
    if (model) model[j] = m;
    for (int t = 0; t < ORC_NP; ++t) {
      double dm = c * wk.dfpp[(size_t)t * P + j];
      if (jac) jac[(size_t)t * P + j] = dm;
      g[t] += wk.w[j] * e * dm;
    }
  }
  for (int t = 0; t < ORC_NP; ++t)
    if (fabs(u[t]) > 1.5) fl |= ORC_OUT_OF_BOX;
  fl |= floor_flag(cfg, u);
  if (fp) memcpy(fp, wk.fp, sizeof(double) * ne);
  if (fpp) memcpy(fpp, wk.fpp, sizeof(double) * P);
  if (b_out) memcpy(b_out, b, sizeof(double) * nd);
  if (chi2) *chi2 = s;
  if (n_eff) *n_eff = wk.n_eff;
  if (grad)
    for (int t = 0; t < ORC_NP; ++t) grad[t] = wk.n_eff > 0 ? -2.0 * g[t] / wk.n_eff : 0.0;
  if (flags) *flags = fl;
  work_free(&wk);
  return rc;
}

/*
 * Weighted residual r_j = sqrt(W_j) (o_j - (P b)_j F''_j) at (u, b), and
 * optionally its Jacobian jac[j][5 + D + 1] with respect to (u, b).
 */
int orc_residual(const orc_cfg *cfg, const float *obs, const float *ivar, const float *basis,
                 const double *u, const double *b, double *r, double *jac) {
  int P = cfg->n_pix, nd = cfg->degree + 1, nx = ORC_NP + nd;
  orc_work wk;
  work_alloc(cfg, &wk);
  setup_data(cfg, obs, ivar, &wk);
  model_spectrum(cfg, basis, u, &wk, jac != NULL);
  for (int j = 0; j < P; ++j) {
    double sw = sqrt(wk.w[j]);
    double c = cont_at(cfg, &wk, b, j);
    r[j] = sw * (wk.o[j] - c * wk.fpp[j]);
    if (jac) {
      for (int t = 0; t < ORC_NP; ++t) jac[(size_t)j * nx + t] = -sw * c * wk.dfpp[(size_t)t * P + j];
      for (int n = 0; n < nd; ++n)
        jac[(size_t)j * nx + ORC_NP + n] = -sw * wk.fpp[j] * wk.leg[(size_t)j * nd + n];
    }
  }
  work_free(&wk);
  return 0;
}

/* Normal matrix N = J^T J and gradient g = J^T r of the weighted residual
 * over the unknowns (u, b); returns chi2 = r^T r. */
static double normal_eq(const orc_cfg *cfg, const orc_work *wk, const double *b, double *N,
                        double *g) {
  int P = cfg->n_pix, nd = cfg->degree + 1, nx = ORC_NP + nd;
  double row[ORC_NP + ORC_DMAX + 1];
  memset(N, 0, sizeof(double) * nx * nx);
  memset(g, 0, sizeof(double) * nx);
  double s = 0.0;
  for (int j = 0; j < P; ++j) {
    if (wk->w[j] == 0.0) continue;
    double sw = sqrt(wk->w[j]);
    double c = cont_at(cfg, wk, b, j);
    double r = sw * (wk->o[j] - c * wk->fpp[j]);
    for (int t = 0; t < ORC_NP; ++t) row[t] = -sw * c * wk->dfpp[(size_t)t * P + j];
    for (int n = 0; n < nd; ++n) row[ORC_NP + n] = -sw * wk->fpp[j] * wk->leg[(size_t)j * nd + n];
    for (int a = 0; a < nx; ++a) {
      g[a] += row[a] * r;
      for (int q = 0; q <= a; ++q) N[a * nx + q] += row[a] * row[q];
    }
    s += r * r;
  }
  for (int a = 0; a < nx; ++a)
    for (int q = a + 1; q < nx; ++q) N[a * nx + q] = N[q * nx + a];
  return s;
}

/*
 * Covariance of the parameters from the final Jacobian: the (u, u) block of
 * s^2 (J^T J)^{-1}, s^2 = chi2 / (n_eff - 5), then mapped to physical units
 * (Teff in K via dTeff = Teff ln10 dlog10 Teff; the others by the box
 * half-widths).  cov_u and cov_phys are 5 x 5 row-major (either may be NULL).
 */
static int covariance(const orc_cfg *cfg, const double *N, double chi2, int n_eff, const double *u,
                      double *cov_u, double *cov_phys) {
  int nd = cfg->degree + 1, nx = ORC_NP + nd;
  double L[(ORC_NP + ORC_DMAX + 1) * (ORC_NP + ORC_DMAX + 1)];
  double inv[(ORC_NP + ORC_DMAX + 1) * (ORC_NP + ORC_DMAX + 1)];
  memcpy(L, N, sizeof(double) * nx * nx);
  int rc = chol(L, nx);
  double s2 = n_eff > ORC_NP ? chi2 / (double)(n_eff - ORC_NP) : NAN;
  double cu[25], cp[25];
  if (rc == 0) {
    chol_inverse(L, nx, inv);
    for (int a = 0; a < ORC_NP; ++a)
      for (int q = 0; q < ORC_NP; ++q) cu[a * 5 + q] = s2 * inv[a * nx + q];
  } else {
    for (int a = 0; a < 25; ++a) cu[a] = NAN;
  }
  double jd[ORC_NP];
  for (int t = 0; t < ORC_NP; ++t) jd[t] = 0.5 * (cfg->hi[t] - cfg->lo[t]);
  double lt = cfg->lo[0] + (u[0] + 1.0) * jd[0];
  jd[0] *= pow(10.0, lt) * ORC_LN10;
  for (int a = 0; a < ORC_NP; ++a)
    for (int q = 0; q < ORC_NP; ++q) cp[a * 5 + q] = jd[a] * cu[a * 5 + q] * jd[q];
  if (cov_u) memcpy(cov_u, cu, sizeof cu);
  if (cov_phys) memcpy(cov_phys, cp, sizeof cp);
  return rc;
}

/*
 * Levenberg-Marquardt fit of one spectrum over (u, b).
 *   u0[5]: start (normalised); b starts at its least-squares value at u0.
 *   Iteration: solve (N + lambda diag(N)) d = -g, accept when chi2 drops
 *   (lambda /= 10), otherwise lambda *= 10 and retry.  Stops after max_iter
 *   accepted or rejected trials, when an accepted step changes u by less
 *   than 1e-12 (max norm), when the relative chi2 drop of an accepted step is
 *   below 1e-14, or when lambda exceeds 1e16.
 * Outputs (each optional): u_out[5], b_out[D+1], chi2, n_eff, cov_u[25],
 * cov_phys[25], n_iter, flags.  Returns 0, or -1 if the normal equations at
 * the start are singular.
 */
int orc_fit(const orc_cfg *cfg, const float *obs, const float *ivar, const float *basis,
            const double *u0, int max_iter, double *u_out, double *b_out, double *chi2_out,
            int *n_eff_out, double *cov_u, double *cov_phys, int *n_iter, unsigned *flags) {
  int nd = cfg->degree + 1, nx = ORC_NP + nd;
  if (nd > ORC_DMAX + 1) return -2;
  orc_work wk;
  work_alloc(cfg, &wk);
  setup_data(cfg, obs, ivar, &wk);
  unsigned fl = wk.flags;
  if (wk.n_eff <= nx) fl |= ORC_NO_DATA;
  double x[ORC_NP + ORC_DMAX + 1], xt[ORC_NP + ORC_DMAX + 1];
  memcpy(x, u0, sizeof(double) * ORC_NP);
  model_spectrum(cfg, basis, x, &wk, 1);
  if (continuum_ls(cfg, &wk, x + ORC_NP) != 0) {
    fl |= ORC_SINGULAR;
    if (flags) *flags = fl;
    work_free(&wk);
    return -1;
  }
  double N[(ORC_NP + ORC_DMAX + 1) * (ORC_NP + ORC_DMAX + 1)];
  double A[(ORC_NP + ORC_DMAX + 1) * (ORC_NP + ORC_DMAX + 1)];
  double g[ORC_NP + ORC_DMAX + 1], d[ORC_NP + ORC_DMAX + 1];
  double chi2 = normal_eq(cfg, &wk, x + ORC_NP, N, g);
  double lambda = 1e-3;
  int it = 0, converged = 0;
  while (it < max_iter) {
    ++it;
    double dmax = 0.0;
    for (int a = 0; a < nx; ++a) dmax = fmax(dmax, N[a * nx + a]);
    memcpy(A, N, sizeof(double) * nx * nx);
    for (int a = 0; a < nx; ++a) A[a * nx + a] += lambda * fmax(N[a * nx + a], 1e-12 * dmax);
    if (chol(A, nx) != 0) {
      lambda *= 10.0;
      if (lambda > 1e16) break;
      continue;
    }
    for (int a = 0; a < nx; ++a) d[a] = -g[a];
    chol_solve(A, nx, d);
    for (int a = 0; a < nx; ++a) xt[a] = x[a] + d[a];
    model_spectrum(cfg, basis, xt, &wk, 0);
    double trial = chi2_at(cfg, &wk, xt + ORC_NP);
    if (isfinite(trial) && trial < chi2) {
      double du = 0.0;
      for (int t = 0; t < ORC_NP; ++t) du = fmax(du, fabs(d[t]));
      double drop = (chi2 - trial) / chi2;
      memcpy(x, xt, sizeof(double) * nx);
      model_spectrum(cfg, basis, x, &wk, 1);
      chi2 = normal_eq(cfg, &wk, x + ORC_NP, N, g);
      lambda = fmax(lambda / 10.0, 1e-15);
      if (du < 1e-12 || drop < 1e-14) {
        converged = 1;
        break;
      }
    } else {
      lambda *= 10.0;
      if (lambda > 1e16) {
        converged = 1; /* no downhill step exists at machine precision */
        break;
      }
    }
  }
  model_spectrum(cfg, basis, x, &wk, 1);
  chi2 = normal_eq(cfg, &wk, x + ORC_NP, N, g);
  if (!converged) fl |= ORC_NOT_CONVERGED;
  for (int t = 0; t < ORC_NP; ++t)
    if (fabs(x[t]) > 1.5) fl |= ORC_OUT_OF_BOX;
  fl |= floor_flag(cfg, x);
  for (int j = 0; j < cfg->n_pix; ++j)
    if (!(cont_at(cfg, &wk, x + ORC_NP, j) > 0.0)) {
      fl |= ORC_CONT_NONPOS;
      break;
    }
  if (covariance(cfg, N, chi2, wk.n_eff, x, cov_u, cov_phys) != 0) fl |= ORC_SINGULAR;
  if (u_out) memcpy(u_out, x, sizeof(double) * ORC_NP);
  if (b_out) memcpy(b_out, x + ORC_NP, sizeof(double) * nd);
  if (chi2_out) *chi2_out = chi2;
  if (n_eff_out) *n_eff_out = wk.n_eff;
  if (n_iter) *n_iter = it;
  if (flags) *flags = fl;
  work_free(&wk);
  return 0;
}

/* Covariance at a given point (u, with b at its least-squares value). */
int orc_covariance(const orc_cfg *cfg, const float *obs, const float *ivar, const float *basis,
                   const double *u, double *cov_u, double *cov_phys) {
  int nd = cfg->degree + 1, nx = ORC_NP + nd;
  orc_work wk;
  work_alloc(cfg, &wk);
  setup_data(cfg, obs, ivar, &wk);
  double x[ORC_NP + ORC_DMAX + 1];
  memcpy(x, u, sizeof(double) * ORC_NP);
  model_spectrum(cfg, basis, x, &wk, 1);
  int rc = continuum_ls(cfg, &wk, x + ORC_NP);
  if (rc == 0) {
    double N[(ORC_NP + ORC_DMAX + 1) * (ORC_NP + ORC_DMAX + 1)], g[ORC_NP + ORC_DMAX + 1];
    double chi2 = normal_eq(cfg, &wk, x + ORC_NP, N, g);
    rc = covariance(cfg, N, chi2, wk.n_eff, x, cov_u, cov_phys);
  }
  (void)nx;
  work_free(&wk);
  return rc;
}

/*
 * Stopping rules of the optimisation stage (Section 2.2, stage 8), for one
 * spectrum.  ell[t] is the loss after t Adam steps (at the parameters the
 * (t+1)-th step would start from).  The per-spectrum loss is the weighted
 * RMS residual sqrt(chi2 / n_eff), the one-spectrum form of Eq. 9.
 * After t steps the fit stops when
 *   rule 2: t >= W and |ell[t-W] - ell[t]| < tol  (the loss changed by less
 *           than tol over the last W steps), or
 *   rule 3: t >= W and ell[s] > ell[s-1] for every s in t-W+1 .. t (the loss
 *           rose at each of the last W steps);
 * rule 1 stops it after n_max steps whatever the loss does.
 * orc_stop_rule tests rules 2 and 3 at one t (ell[0..t] known) and returns
 * 2, 3 or 0.  orc_stop_step scans t = 0 .. n_max - 1 and returns the first
 * t at which rule 2 or 3 holds, with the rule in *rule; otherwise n_max
 * with *rule = 1.  Rule 2 is tested first.
 */
int orc_clean(int n, const float *obs, const float *ivar, const double *model, double f_shift,
              unsigned char *keep, double *k_used, int *d_iters);

int orc_stop_rule(const double *ell, int t, int W, double tol) {
  if (W <= 0 || t < W) return 0;
  if (fabs(ell[t - W] - ell[t]) < tol) return 2;
  for (int q = t - W + 1; q <= t; ++q)
    if (!(ell[q] > ell[q - 1])) return 0;
  return 3;
}

int orc_stop_step(const double *ell, int n_max, int W, double tol, int *rule) {
  for (int t = 0; t < n_max; ++t) {
    int r = orc_stop_rule(ell, t, W, tol);
    if (r) {
      if (rule) *rule = r;
      return t;
    }
  }
  if (rule) *rule = 1;
  return n_max;
}

/*
 * The paper's optimiser for one spectrum: Adam (Kingma & Ba) on
 * J = chi2 / n_eff over the normalised parameters u, each step using the
 * gradient of orc_eval (continuum at its least-squares value), in the form
 * of torch.optim.Adam with default settings other than lr: m and v are the
 * first and second moment estimates, bias corrected with beta^t, and eps is
 * added to the square root of the corrected v.  With W > 0 the stopping
 * rules above end the fit (the step that would follow is not taken).
 * With clean_every > 0 the Clean strategy of stage 8 updates the mask after
 * every clean_every steps, at most clean_max times: the model at the
 * current parameters gives the residuals, orc_clean gives the mask (f_shift
 * 0.5 at the first update, 0.2 after), and masked pixels get weight zero
 * from then on (each update starts from the input weights).
 * Outputs: u_out[5], steps taken, rule (1, 2, 3), and optionally
 * ell_out[0..steps] (n_max + 1 entries) and keep_out[P] (final mask).
 * Returns 0.
 */
int orc_adam_fit(const orc_cfg *cfg, const float *obs, const float *ivar, const float *basis,
                 const double *u0, int n_max, double lr, double beta1, double beta2, double eps,
                 int W, double tol, int clean_every, int clean_max, double *u_out,
                 int *steps_out, int *rule_out, double *ell_out, unsigned char *keep_out) {
  double u[ORC_NP], m[ORC_NP] = {0, 0, 0, 0, 0}, v[ORC_NP] = {0, 0, 0, 0, 0};
  memcpy(u, u0, sizeof(u));
  const int P = cfg->n_pix;
  double *ell = (double *)malloc(sizeof(double) * (size_t)(n_max + 1));
  float *iv = (float *)malloc(sizeof(float) * (size_t)P);
  double *model = (double *)malloc(sizeof(double) * (size_t)P);
  unsigned char *keep = (unsigned char *)malloc((size_t)P);
  memcpy(iv, ivar, sizeof(float) * (size_t)P);
  memset(keep, 1, (size_t)P);
  int t = 0, rule = 1, updates = 0;
  for (;; ++t) {
    if (clean_every > 0 && t > 0 && t % clean_every == 0 && updates < clean_max) {
      orc_eval(cfg, obs, ivar, basis, u, NULL, NULL, NULL, model, NULL, NULL, NULL, NULL, NULL);
      orc_clean(P, obs, ivar, model, updates == 0 ? 0.5 : 0.2, keep, NULL, NULL);
      for (int j = 0; j < P; ++j) iv[j] = keep[j] ? ivar[j] : 0.0f;
      ++updates;
    }
    double chi2 = 0.0, g[ORC_NP];
    int n_eff = 0;
    orc_eval(cfg, obs, iv, basis, u, NULL, NULL, NULL, NULL, &chi2, &n_eff, g, NULL, NULL);
    ell[t] = n_eff > 0 ? sqrt(chi2 / (double)n_eff) : 0.0;
    if (t == n_max) break;
    int r = orc_stop_rule(ell, t, W, tol);
    if (r) {
      rule = r;
      break;
    }
    const int step = t + 1;
    const double bc1 = 1.0 - pow(beta1, (double)step);
    const double bc2 = 1.0 - pow(beta2, (double)step);
    for (int a = 0; a < ORC_NP; ++a) {
      m[a] = beta1 * m[a] + (1.0 - beta1) * g[a];
      v[a] = beta2 * v[a] + (1.0 - beta2) * g[a] * g[a];
      u[a] -= lr * (m[a] / bc1) / (sqrt(v[a] / bc2) + eps);
    }
  }
  memcpy(u_out, u, sizeof(u));
  if (steps_out) *steps_out = t;
  if (rule_out) *rule_out = rule;
  if (ell_out) memcpy(ell_out, ell, sizeof(double) * (size_t)(t + 1));
  if (keep_out) memcpy(keep_out, keep, (size_t)P);
  free(ell);
  free(iv);
  free(model);
  free(keep);
  return 0;
}

/*
 * Clean outlier mask of one spectrum (Section 2.2, step 6, the three-step
 * clipping of the Clean strategy), from its residual eps = o - m against a
 * model m and its valid pixels (W > 0).  Readings: sigma is the sample
 * standard deviation (n - 1) of eps over the valid pixels; sigma' in the
 * third step uses the valid pixels kept by the first two steps; the flux
 * gradient G_j = max(|m_j - m_{j-1}|, |m_j - m_{j+1}|) uses the neighbour
 * that exists at the ends of the spectrum; only valid pixels are tested and
 * only valid pixels seed a neighbour test.
 *   B: |eps_j| - f G_j > k sigma masks j; k = 3, relaxed to 4, 5, 7 while
 *      more than 3 % of the valid pixels would be masked.
 *   C: a neighbour j' of a B outlier with |eps_j'| - f G_j' > 2 sigma.
 *   D: a neighbour j' of an outlier j (B, C or D) with eps_j eps_j' > 0,
 *      |eps_j'| <= |eps_j| and |eps_j'| - f G_j' > sigma'; repeated until D
 *      does not change, at most 20 times.
 * keep[j] = 1 if kept (A_j = B_j C_j D_j = 1), 0 if masked; invalid pixels
 * are reported as kept (they carry no weight).  Returns the number of
 * masked valid pixels; *k_used gets the accepted k, *d_iters the D passes.
 */
int orc_clean(int n, const float *obs, const float *ivar, const double *model, double f_shift,
              unsigned char *keep, double *k_used, int *d_iters) {
  unsigned char *valid = (unsigned char *)malloc((size_t)n);
  unsigned char *B = (unsigned char *)malloc((size_t)n);
  unsigned char *C = (unsigned char *)malloc((size_t)n);
  unsigned char *D = (unsigned char *)malloc((size_t)n);
  unsigned char *Dn = (unsigned char *)malloc((size_t)n);
  double *eps = (double *)malloc(sizeof(double) * (size_t)n);
  double *G = (double *)malloc(sizeof(double) * (size_t)n);
  int nv = 0;
  for (int j = 0; j < n; ++j) {
    valid[j] = isfinite(obs[j]) && isfinite(ivar[j]) && ivar[j] > 0.0f;
    eps[j] = (double)obs[j] - model[j];
    double gl = j > 0 ? fabs(model[j] - model[j - 1]) : 0.0;
    double gr = j + 1 < n ? fabs(model[j] - model[j + 1]) : 0.0;
    G[j] = gl > gr ? gl : gr;
    nv += valid[j];
    B[j] = C[j] = D[j] = 1;
  }
  double mean = 0.0, var = 0.0;
  for (int j = 0; j < n; ++j)
    if (valid[j]) mean += eps[j];
  mean = nv > 0 ? mean / nv : 0.0;
  for (int j = 0; j < n; ++j)
    if (valid[j]) var += (eps[j] - mean) * (eps[j] - mean);
  const double sigma = nv > 1 ? sqrt(var / (nv - 1)) : 0.0;
  /* step B with the relaxed thresholds */
  static const double ks[4] = {3.0, 4.0, 5.0, 7.0};
  double k = 7.0;
  for (int q = 0; q < 4; ++q) {
    int cnt = 0;
    for (int j = 0; j < n; ++j)
      if (valid[j] && fabs(eps[j]) - f_shift * G[j] > ks[q] * sigma) ++cnt;
    if (cnt <= 0.03 * nv || q == 3) {
      k = ks[q];
      break;
    }
  }
  for (int j = 0; j < n; ++j)
    B[j] = !(valid[j] && fabs(eps[j]) - f_shift * G[j] > k * sigma);
  /* step C */
  for (int j = 0; j < n; ++j) {
    if (B[j]) continue;
    for (int s = -1; s <= 1; s += 2) {
      int jp = j + s;
      if (jp < 0 || jp >= n || !valid[jp]) continue;
      if (fabs(eps[jp]) - f_shift * G[jp] > 2.0 * sigma) C[jp] = 0;
    }
  }
  /* sigma' over the valid pixels kept by B and C */
  int n2 = 0;
  double mean2 = 0.0, var2 = 0.0;
  for (int j = 0; j < n; ++j)
    if (valid[j] && B[j] && C[j]) {
      mean2 += eps[j];
      ++n2;
    }
  mean2 = n2 > 0 ? mean2 / n2 : 0.0;
  for (int j = 0; j < n; ++j)
    if (valid[j] && B[j] && C[j]) var2 += (eps[j] - mean2) * (eps[j] - mean2);
  const double sigma2 = n2 > 1 ? sqrt(var2 / (n2 - 1)) : 0.0;
  /* step D, repeated until it does not change */
  int it = 0;
  for (; it < 20; ++it) {
    memcpy(Dn, D, (size_t)n);
    for (int j = 0; j < n; ++j) {
      if (!valid[j] || (B[j] && C[j] && D[j])) continue;
      for (int s = -1; s <= 1; s += 2) {
        int jp = j + s;
        if (jp < 0 || jp >= n || !valid[jp]) continue;
        if (eps[j] * eps[jp] > 0.0 && fabs(eps[jp]) <= fabs(eps[j]) &&
            fabs(eps[jp]) - f_shift * G[jp] > sigma2)
          Dn[jp] = 0;
      }
    }
    int changed = memcmp(Dn, D, (size_t)n) != 0;
    memcpy(D, Dn, (size_t)n);
    if (!changed) break;
  }
  int masked = 0;
  for (int j = 0; j < n; ++j) {
    keep[j] = !(valid[j] && !(B[j] && C[j] && D[j]));
    masked += !keep[j];
  }
  if (k_used) *k_used = k;
  if (d_iters) *d_iters = it;
  free(valid); free(B); free(C); free(D); free(Dn); free(eps); free(G);
  return masked;
}

/*
 * Flux-conserving resampling (Section 2.2, step 3) of one spectrum from a
 * linear wavelength grid (bin centres lam0 + i dlam, i < n_src) onto a
 * logarithmic grid of n_out pixels with centres 10^(lg0 + j dlog10), in the
 * paper's four steps:
 *   1. integration nodes: the source bin edges lam0 - dlam/2 + k dlam and
 *      the target edges 10^(lg0 + (j - 1/2) dlog10), j = 0..n_out;
 *   2. the cumulative integral of the source at its nodes, 0, T_1 dlam,
 *      (T_1 + T_2) dlam, ...;
 *   3. that integral interpolated linearly at the target nodes (constant
 *      beyond the source range);
 *   4. the differences of step 3 divided by the target bin widths.
 * Reading: base 10 (the grid of the paper's Section 4), as for the model.
 * out[j] in FP64.  Returns 0, or -1 if the target range leaves the source.
 */
int orc_resample(int n_src, double lam0, double dlam, const float *src, int n_out, double lg0,
                 double dlog10, double *out) {
  double *cum = (double *)malloc(sizeof(double) * (size_t)(n_src + 1));
  cum[0] = 0.0;
  for (int k = 0; k < n_src; ++k) cum[k + 1] = cum[k] + (double)src[k] * dlam;
  const double e0 = lam0 - 0.5 * dlam;
  const double e_end = e0 + n_src * dlam;
  int rc = 0;
  double prev_l = 0.0, prev_f = 0.0;
  for (int j = 0; j <= n_out; ++j) {
    const double l = pow(10.0, lg0 + ((double)j - 0.5) * dlog10);
    if (l < e0 || l > e_end) rc = -1;
    double f;
    if (l <= e0) {
      f = 0.0;
    } else if (l >= e_end) {
      f = cum[n_src];
    } else {
      int k = (int)floor((l - e0) / dlam);
      if (k > n_src - 1) k = n_src - 1;
      const double frac = (l - (e0 + k * dlam)) / dlam;
      f = cum[k] + frac * (cum[k + 1] - cum[k]);
    }
    if (j > 0) out[j - 1] = (f - prev_f) / (l - prev_l);
    prev_l = l;
    prev_f = f;
  }
  free(cum);
  return rc;
}
