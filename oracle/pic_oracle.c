/*
 * pic_oracle.c -- plain, single-threaded FP64 reference of one electromagnetic
 * PIC step for relativistic beams (Xu et al., "On numerical errors to the
 * fields surrounding a relativistically moving particle in PIC codes").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code with
 * the GPU path and is written for clarity, not speed: every loop runs over
 * plain arrays in the order the method states it.
 *
 * What one step computes (Sec. 1 PIC cycle; Sec. 2.1 Eq. 1; Eq. 14 Yee
 * operators; App. C customized axial operator):
 *   1. gather E^n, B^n at x^n with the quadratic B-spline shape, each
 *      staggered component with weights taken at its own lattice points;
 *   2. relativistic Boris rotation  u^{n-1/2} -> u^{n+1/2};
 *   3. x^{n+1} = x^n + dt u^{n+1/2} / gamma^{n+1/2};
 *   4. charge-conserving current J^{n+1/2} (Esirkepov's density decomposition
 *      for the quadratic spline), so the discrete continuity equation holds
 *      with the Yee divergence (Sec. 2.1: Gauss is kept by charge
 *      conservation);
 *   5. customized solver only: J1 <- G * J1 along x1 where G inverts the
 *      telescoped stencil K (d-_custom = K * d-_Yee), so continuity also holds
 *      with the customized divergence (Sec. 3, current correction);
 *   6. B^{n+1/2} = B^n - dt/2 d+ x E^n;  E^{n+1} = E^n + dt (d- x B^{n+1/2} - J);
 *      B^{n+1} = B^{n+1/2} - dt/2 d+ x E^{n+1}   (leapfrog, [omega]_t of Sec. 2.1);
 *   7. moving window: shift one cell when the window edge crosses a cell.
 *
 * Units: c = 1, d_t E = curl B - J, div E = rho (Eqs. 1 and 5).  Lengths are in
 * cells for particle positions; dx, dt are physical.
 *
 * Yee lattice (node = integer index):  E1 (i1+1/2,i2,i3)  E2 (i1,i2+1/2,i3)
 * E3 (i1,i2,i3+1/2)  B1 (i1,i2+1/2,i3+1/2)  B2 (i1+1/2,i2,i3+1/2)
 * B3 (i1+1/2,i2+1/2,i3);  J like E; rho at nodes.  In 2D the i3 coordinate is
 * dropped and all d/dx3 vanish.
 *
 * Axial operators (App. C, the two one-sided forms):
 *   d+ f_i = (1/dx1) sum_{l=1..M} C_l  (f_{i+l}   - f_{i-l+1})   acts on E -> B
 *   d- f_i = (1/dx1) sum_{l=1..M} CB_l (f_{i+l-1} - f_{i-l})     acts on B -> E
 * M = 1, C_1 = 1 is the Yee operator.  x2 and x3 always use the Yee form.
 * CB defaults to C ([k]_E1 = [k]_B1, Sec. 3's choice); Sec. 3 also allows
 * [k]_E1 != [k]_B1 with [k]_E1 [k]_B1 = [k1]_t^2, e.g. [k]_B1 = Yee.  d- is
 * the operator of Ampere's law and therefore of Gauss's law and of the
 * continuity equation, so the J1 correction follows CB.
 *
 * Threads (OpenMP, optional): only loops whose iterations write disjoint
 * results run in parallel -- the field updates cell by cell, the J1
 * correction line by line, and the gather + push particle by particle.  The
 * current deposit (a sum over particles into shared nodes) and every
 * reduction run serially in a fixed order, so the results do not depend on
 * the number of threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXM 64
#define ORC_PI 3.14159265358979323846

typedef struct {
  int ndim;
  long n[3];
  double dx[3];
  double dt;
  int window;   /* 0: periodic in x1;  1: moving window along +x1 */
  double vwin;  /* window speed in units of c */
  int M;
  double C[ORC_MAXM];   /* d+ (E -> B) */
  double CB[ORC_MAXM];  /* d- (B -> E), zero-padded to M */
  int correct;  /* apply the J1 correction (customized d-) */
  long N;       /* number of cells */
  double *F[9]; /* E1 E2 E3 B1 B2 B3 J1 J2 J3 */
  /* particles: absolute positions in cell units (x1 is the global index) */
  long np, cap;
  double *x[3], *u[3], *Q, *qm;
  int *alive;
  long ws;    /* global x1 index of the first window cell */
  long step;  /* completed steps */
  /* J1 correction kernel: g[j] for j in [-ng, ng] stored at g[j + ng] */
  double *g;
  long ng;
  int g_circular;
  /* current smoothing along x1 (0 passes: off) */
  int filt_npass;
  double filt_comp;
  /* plasma injection at window shifts */
  int inj_on;
  int inj_ppc[3];
  double inj_Q, inj_qm, inj_uth;
  uint64_t inj_seed;
  long inj_count; /* particles injected so far: counter for the generator */
} orc_sim;

#define E1 0
#define E2 1
#define E3 2
#define B1 3
#define B2 4
#define B3 5
#define J1 6
#define J2 7
#define J3 8

static long wrapl(long i, long n) {
  long r = i % n;
  return r < 0 ? r + n : r;
}

/* field value at lattice index (i1 logical within the window), with the
 * boundary rule: x2, x3 periodic; x1 periodic, or zero outside the window */
static double fget(const orc_sim *s, const double *f, long i1, long i2, long i3) {
  if (s->window) {
    if (i1 < 0 || i1 >= s->n[0]) return 0.0;
  } else {
    i1 = wrapl(i1, s->n[0]);
  }
  i2 = wrapl(i2, s->n[1]);
  i3 = wrapl(i3, s->n[2]);
  return f[i1 + s->n[0] * (i2 + s->n[1] * i3)];
}

static double *fref(orc_sim *s, double *f, long i1, long i2, long i3) {
  if (s->window) {
    if (i1 < 0 || i1 >= s->n[0]) return NULL;
  } else {
    i1 = wrapl(i1, s->n[0]);
  }
  i2 = wrapl(i2, s->n[1]);
  i3 = wrapl(i3, s->n[2]);
  return &f[i1 + s->n[0] * (i2 + s->n[1] * i3)];
}

/* axial forward / backward differences (App. C) */
static double d1p(const orc_sim *s, const double *f, long i1, long i2, long i3) {
  double acc = 0.0;
  for (int l = 1; l <= s->M; ++l)
    acc += s->C[l - 1] * (fget(s, f, i1 + l, i2, i3) - fget(s, f, i1 - l + 1, i2, i3));
  return acc / s->dx[0];
}
static double d1m(const orc_sim *s, const double *f, long i1, long i2, long i3) {
  double acc = 0.0;
  for (int l = 1; l <= s->M; ++l)
    acc += s->CB[l - 1] * (fget(s, f, i1 + l - 1, i2, i3) - fget(s, f, i1 - l, i2, i3));
  return acc / s->dx[0];
}
/* transverse Yee differences (Eq. 14) */
static double d2p(const orc_sim *s, const double *f, long i1, long i2, long i3) {
  return (fget(s, f, i1, i2 + 1, i3) - fget(s, f, i1, i2, i3)) / s->dx[1];
}
static double d2m(const orc_sim *s, const double *f, long i1, long i2, long i3) {
  return (fget(s, f, i1, i2, i3) - fget(s, f, i1, i2 - 1, i3)) / s->dx[1];
}
static double d3p(const orc_sim *s, const double *f, long i1, long i2, long i3) {
  if (s->ndim < 3) return 0.0;
  return (fget(s, f, i1, i2, i3 + 1) - fget(s, f, i1, i2, i3)) / s->dx[2];
}
static double d3m(const orc_sim *s, const double *f, long i1, long i2, long i3) {
  if (s->ndim < 3) return 0.0;
  return (fget(s, f, i1, i2, i3) - fget(s, f, i1, i2, i3 - 1)) / s->dx[2];
}

/* quadratic B-spline of a distance measured in cells */
static double spline2(double d) {
  d = fabs(d);
  if (d <= 0.5) return 0.75 - d * d;
  if (d < 1.5) {
    double t = 1.5 - d;
    return 0.5 * t * t;
  }
  return 0.0;
}

/* K^(theta) = [k]_B1 / [k]_Yee, the symbol of the telescoped d- stencil */
static double khat_ratio(const orc_sim *s, double th) {
  double num = 0.0, den = sin(0.5 * th);
  if (fabs(den) < 1e-300) {
    double lim = 0.0;
    for (int l = 1; l <= s->M; ++l) lim += s->CB[l - 1] * (2.0 * l - 1.0);
    return lim;
  }
  for (int l = 1; l <= s->M; ++l) num += s->CB[l - 1] * sin((2.0 * l - 1.0) * 0.5 * th);
  return num / den;
}

/* G = 1/K^ sampled on an Nq-point periodic grid and transformed back:
 * g_j = (1/Nq) sum_m cos(2 pi m j / Nq) / K^(2 pi m / Nq).  For a periodic x1
 * line of length N1 this is the exact circulant inverse (Nq = N1).  For the
 * moving window, Nq is large and g_j is the infinite-line inverse to
 * round-off; it is applied with zero extension and cut where
 * |g_j| < 1e-16 |g_0| (its terms are then at FP64 round-off of the leading
 * tap; the DFT sum itself has a noise floor near 1e-17). */
static void build_correction(orc_sim *s) {
  free(s->g);
  s->g = NULL;
  s->ng = 0;
  if (!s->correct) return;
  long Nq = s->window ? 16384 : s->n[0];
  double *inv = (double *)malloc(sizeof(double) * Nq);
  for (long m = 0; m < Nq; ++m) inv[m] = 1.0 / khat_ratio(s, 2.0 * ORC_PI * (double)m / (double)Nq);
  /* taps j = 0..half (g is even in j) */
  long half = s->window ? (s->n[0] - 1) : (Nq - 1);
  double *gj = (double *)malloc(sizeof(double) * (half + 1));
  for (long j = 0; j <= half; ++j) {
    double acc = 0.0;
    for (long m = 0; m < Nq; ++m) acc += cos(2.0 * ORC_PI * (double)((m * j) % Nq) / (double)Nq) * inv[m];
    gj[j] = acc / (double)Nq;
  }
  free(inv);
  if (s->window) {
    long cut = half;
    while (cut > 0 && fabs(gj[cut]) < 1e-16 * fabs(gj[0])) --cut;
    s->ng = cut;
    s->g = (double *)malloc(sizeof(double) * (2 * cut + 1));
    for (long j = -cut; j <= cut; ++j) s->g[j + cut] = gj[labs(j)];
    s->g_circular = 0;
    free(gj);
  } else {
    /* circulant inverse on the periodic line: g[j], j = 0..N1-1 */
    s->g = gj;
    s->g_circular = 1;
  }
}

void *orc_create(int ndim, const long *n, const double *dx, double dt, int window,
                 double vwin, int M, const double *C, int MB, const double *CB, int correct) {
  if (ndim < 2 || ndim > 3 || M < 1 || M > ORC_MAXM || MB < 0 || MB > ORC_MAXM) return NULL;
  orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
  s->ndim = ndim;
  for (int d = 0; d < 3; ++d) {
    s->n[d] = (d < ndim) ? n[d] : 1;
    s->dx[d] = (d < ndim) ? dx[d] : 1.0;
  }
  s->dt = dt;
  s->window = window;
  s->vwin = vwin;
  /* both operators on max(M, MB) coefficients, the shorter one zero-padded */
  int Mx = (MB > M) ? MB : M;
  s->M = Mx;
  for (int l = 0; l < Mx; ++l) {
    s->C[l] = (l < M) ? C[l] : 0.0;
    s->CB[l] = (MB == 0) ? s->C[l] : ((l < MB) ? CB[l] : 0.0);
  }
  s->correct = correct;
  s->N = s->n[0] * s->n[1] * s->n[2];
  for (int k = 0; k < 9; ++k) s->F[k] = (double *)calloc((size_t)s->N, sizeof(double));
  build_correction(s);
  return s;
}

void orc_destroy(void *h) {
  orc_sim *s = (orc_sim *)h;
  if (!s) return;
  for (int k = 0; k < 9; ++k) free(s->F[k]);
  for (int d = 0; d < 3; ++d) {
    free(s->x[d]);
    free(s->u[d]);
  }
  free(s->Q);
  free(s->qm);
  free(s->alive);
  free(s->g);
  free(s);
}

static void grow(orc_sim *s, long need) {
  if (need <= s->cap) return;
  long cap = s->cap ? s->cap : 16;
  while (cap < need) cap *= 2;
  for (int d = 0; d < 3; ++d) {
    s->x[d] = (double *)realloc(s->x[d], sizeof(double) * cap);
    s->u[d] = (double *)realloc(s->u[d], sizeof(double) * cap);
  }
  s->Q = (double *)realloc(s->Q, sizeof(double) * cap);
  s->qm = (double *)realloc(s->qm, sizeof(double) * cap);
  s->alive = (int *)realloc(s->alive, sizeof(int) * cap);
  s->cap = cap;
}

/* x: [np][ndim] positions in cell units (x1 global); u: [np][3] = gamma*beta.
 * Q: charge of one macro-particle, qm: charge/mass of the species. */
long orc_add_particles(void *h, long np, const double *x, const double *u, double Q, double qm) {
  orc_sim *s = (orc_sim *)h;
  grow(s, s->np + np);
  for (long p = 0; p < np; ++p) {
    long k = s->np + p;
    for (int d = 0; d < 3; ++d) {
      s->x[d][k] = (d < s->ndim) ? x[p * s->ndim + d] : 0.0;
      s->u[d][k] = u[p * 3 + d];
    }
    s->Q[k] = Q;
    s->qm[k] = qm;
    s->alive[k] = 1;
  }
  s->np += np;
  return s->np;
}

/* E or B component at a particle position x (cell units, x1 global).  Each
 * component is interpolated from its own staggered points with the quadratic
 * spline; stag[d] = 1 where the component sits at half-integer points. */
static double interp(const orc_sim *s, const double *f, const int *stag, const double *x) {
  double acc = 0.0;
  long lo[3], hi[3];
  for (int d = 0; d < 3; ++d) {
    if (d < s->ndim) {
      long c = (long)floor(x[d]);
      lo[d] = c - 2;
      hi[d] = c + 2;
    } else {
      lo[d] = hi[d] = 0;
    }
  }
  for (long k = lo[2]; k <= hi[2]; ++k) {
    double w3 = (s->ndim == 3) ? spline2((double)k + 0.5 * stag[2] - x[2]) : 1.0;
    if (w3 == 0.0) continue;
    for (long j = lo[1]; j <= hi[1]; ++j) {
      double w2 = spline2((double)j + 0.5 * stag[1] - x[1]);
      if (w2 == 0.0) continue;
      for (long i = lo[0]; i <= hi[0]; ++i) {
        double w1 = spline2((double)i + 0.5 * stag[0] - x[0]);
        if (w1 == 0.0) continue;
        acc += w1 * w2 * w3 * fget(s, f, i - s->ws, j, k);
      }
    }
  }
  return acc;
}

static const int STAG[6][3] = {
    {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, /* E1 E2 E3 */
    {0, 1, 1}, {1, 0, 1}, {1, 1, 0}, /* B1 B2 B3 */
};

static void gather(const orc_sim *s, const double *x, double *EB) {
  for (int c = 0; c < 6; ++c) {
    int st[3] = {STAG[c][0], STAG[c][1], STAG[c][2]};
    if (s->ndim == 2) st[2] = 0;
    EB[c] = interp(s, s->F[c], st, x);
  }
}

/* E and B interpolated at arbitrary positions (for self-force diagnostics) */
void orc_gather_at(void *h, long npts, const double *x, double *EB) {
  orc_sim *s = (orc_sim *)h;
  for (long p = 0; p < npts; ++p) {
    double xx[3] = {0, 0, 0};
    for (int d = 0; d < s->ndim; ++d) xx[d] = x[p * s->ndim + d];
    gather(s, xx, &EB[6 * p]);
  }
}

/* relativistic Boris push (textbook form): half electric kick, magnetic
 * rotation with t = (q dt / 2m) B / gamma, s = 2t / (1 + t^2), half kick */
static void boris(double qm, double dt, const double *EB, double *u) {
  double a = 0.5 * qm * dt;
  double um[3], t[3], sv[3], up[3], upl[3];
  for (int d = 0; d < 3; ++d) um[d] = u[d] + a * EB[d];
  double g = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
  for (int d = 0; d < 3; ++d) t[d] = a * EB[3 + d] / g;
  double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
  for (int d = 0; d < 3; ++d) sv[d] = 2.0 * t[d] / (1.0 + t2);
  up[0] = um[0] + (um[1] * t[2] - um[2] * t[1]);
  up[1] = um[1] + (um[2] * t[0] - um[0] * t[2]);
  up[2] = um[2] + (um[0] * t[1] - um[1] * t[0]);
  upl[0] = um[0] + (up[1] * sv[2] - up[2] * sv[1]);
  upl[1] = um[1] + (up[2] * sv[0] - up[0] * sv[2]);
  upl[2] = um[2] + (up[0] * sv[1] - up[1] * sv[0]);
  for (int d = 0; d < 3; ++d) u[d] = upl[d] + a * EB[d];
}

static void add_j(orc_sim *s, int comp, long i1g, long i2, long i3, double v) {
  double *r = fref(s, s->F[comp], i1g - s->ws, i2, i3);
  if (r) *r += v;
}

/* Esirkepov current for one particle moving xo -> xn (cell units).  The
 * density change is split into W1 + W2 (+ W3) with
 *   2D: W1 = DS1 (S2 + DS2/2),  W2 = DS2 (S1 + DS1/2)
 *   3D: W1 = DS1 (S2 S3 + DS2 S3/2 + S2 DS3/2 + DS2 DS3/3)  (and cyclic)
 * and J_d at half points is minus the running sum of W_d along d, times
 * Q dx_d / (dV dt).  In 2D the out-of-plane current is Q v3 W3 / dV with
 * W3 = S1 S2 + DS1 S2/2 + S1 DS2/2 + DS1 DS2/3. */
static void deposit(orc_sim *s, double Q, const double *xo, const double *xn, double v3) {
  int nd = s->ndim;
  long base[3] = {0, 0, 0};
  double S0[3][5], DS[3][5];
  double dV = s->dx[0] * s->dx[1] * (nd == 3 ? s->dx[2] : 1.0);
  for (int d = 0; d < 3; ++d) {
    for (int k = 0; k < 5; ++k) {
      S0[d][k] = (k == 2) ? 1.0 : 0.0;
      DS[d][k] = 0.0;
    }
  }
  for (int d = 0; d < nd; ++d) {
    base[d] = (long)floor(xo[d] + 0.5);
    for (int k = 0; k < 5; ++k) {
      double node = (double)(base[d] + k - 2);
      S0[d][k] = spline2(node - xo[d]);
      DS[d][k] = spline2(node - xn[d]) - S0[d][k];
    }
  }
  double f1 = -Q * s->dx[0] / (dV * s->dt);
  double f2 = -Q * s->dx[1] / (dV * s->dt);
  if (nd == 2) {
    for (int b = 0; b < 5; ++b) {
      double run = 0.0;
      for (int a = 0; a < 5; ++a) {
        run += DS[0][a] * (S0[1][b] + 0.5 * DS[1][b]);
        if (run != 0.0) add_j(s, J1, base[0] + a - 2, base[1] + b - 2, 0, f1 * run);
      }
    }
    for (int a = 0; a < 5; ++a) {
      double run = 0.0;
      for (int b = 0; b < 5; ++b) {
        run += DS[1][b] * (S0[0][a] + 0.5 * DS[0][a]);
        if (run != 0.0) add_j(s, J2, base[0] + a - 2, base[1] + b - 2, 0, f2 * run);
      }
    }
    for (int a = 0; a < 5; ++a)
      for (int b = 0; b < 5; ++b) {
        double w3 = S0[0][a] * S0[1][b] + 0.5 * DS[0][a] * S0[1][b] + 0.5 * S0[0][a] * DS[1][b] +
                    DS[0][a] * DS[1][b] / 3.0;
        if (w3 != 0.0) add_j(s, J3, base[0] + a - 2, base[1] + b - 2, 0, Q * v3 * w3 / dV);
      }
    return;
  }
  double f3 = -Q * s->dx[2] / (dV * s->dt);
  /* J1 */
  for (int c = 0; c < 5; ++c)
    for (int b = 0; b < 5; ++b) {
      double run = 0.0;
      for (int a = 0; a < 5; ++a) {
        run += DS[0][a] * (S0[1][b] * S0[2][c] + 0.5 * DS[1][b] * S0[2][c] + 0.5 * S0[1][b] * DS[2][c] +
                           DS[1][b] * DS[2][c] / 3.0);
        if (run != 0.0) add_j(s, J1, base[0] + a - 2, base[1] + b - 2, base[2] + c - 2, f1 * run);
      }
    }
  /* J2 */
  for (int c = 0; c < 5; ++c)
    for (int a = 0; a < 5; ++a) {
      double run = 0.0;
      for (int b = 0; b < 5; ++b) {
        run += DS[1][b] * (S0[0][a] * S0[2][c] + 0.5 * DS[0][a] * S0[2][c] + 0.5 * S0[0][a] * DS[2][c] +
                           DS[0][a] * DS[2][c] / 3.0);
        if (run != 0.0) add_j(s, J2, base[0] + a - 2, base[1] + b - 2, base[2] + c - 2, f2 * run);
      }
    }
  /* J3 */
  for (int b = 0; b < 5; ++b)
    for (int a = 0; a < 5; ++a) {
      double run = 0.0;
      for (int c = 0; c < 5; ++c) {
        run += DS[2][c] * (S0[0][a] * S0[1][b] + 0.5 * DS[0][a] * S0[1][b] + 0.5 * S0[0][a] * DS[1][b] +
                           DS[0][a] * DS[1][b] / 3.0);
        if (run != 0.0) add_j(s, J3, base[0] + a - 2, base[1] + b - 2, base[2] + c - 2, f3 * run);
      }
    }
}

static void correct_j1(orc_sim *s) {
  long n1 = s->n[0];
  long nlines = s->n[1] * s->n[2];
#pragma omp parallel
  {
    double *line = (double *)malloc(sizeof(double) * n1);
    double *out = (double *)malloc(sizeof(double) * n1);
#pragma omp for schedule(dynamic, 16)
    for (long ln = 0; ln < nlines; ++ln) {
      double *f = &s->F[J1][n1 * ln];
      int nz = 0;
      for (long i = 0; i < n1; ++i) {
        line[i] = f[i];
        if (f[i] != 0.0) nz = 1;
      }
      if (!nz) continue;
      for (long i = 0; i < n1; ++i) {
        double acc = 0.0;
        if (s->g_circular) {
          for (long m = 0; m < n1; ++m) acc += s->g[m] * line[wrapl(i - m, n1)];
        } else {
          for (long m = -s->ng; m <= s->ng; ++m) {
            long src = i - m;
            if (src >= 0 && src < n1) acc += s->g[m + s->ng] * line[src];
          }
        }
        out[i] = acc;
      }
      for (long i = 0; i < n1; ++i) f[i] = out[i];
    }
    free(line);
    free(out);
  }
}

/* Smoothing of the current along x1: npass binomial passes (1, 2, 1)/4 and
 * one compensator pass (-c/4, 1 + c/2, -c/4), symbol
 * cos^(2 npass)(k dx1/2) (1 + c sin^2(k dx1/2)).  x1 is periodic, or zero
 * beyond the moving window.  Every component gets the same x1 filter, which
 * commutes with the divergence, so Gauss's law holds for the filtered
 * density. */
static void filter_line(double *f, double *tmp, long n1, int window, double a, double b) {
  for (long i = 0; i < n1; ++i) {
    double lo, hi;
    if (window) {
      lo = (i > 0) ? f[i - 1] : 0.0;
      hi = (i < n1 - 1) ? f[i + 1] : 0.0;
    } else {
      lo = f[wrapl(i - 1, n1)];
      hi = f[wrapl(i + 1, n1)];
    }
    tmp[i] = a * lo + b * f[i] + a * hi;
  }
  for (long i = 0; i < n1; ++i) f[i] = tmp[i];
}

static void filter_j(orc_sim *s) {
  long n1 = s->n[0];
  long nlines = s->n[1] * s->n[2];
#pragma omp parallel
  {
    double *tmp = (double *)malloc(sizeof(double) * n1);
#pragma omp for schedule(static)
    for (long ln = 0; ln < nlines; ++ln)
      for (int c = J1; c <= J3; ++c) {
        double *f = &s->F[c][n1 * ln];
        for (int p = 0; p < s->filt_npass; ++p) filter_line(f, tmp, n1, s->window, 0.25, 0.5);
        filter_line(f, tmp, n1, s->window, -0.25 * s->filt_comp, 1.0 + 0.5 * s->filt_comp);
      }
    free(tmp);
  }
}

void orc_set_filter(void *h, int npass, double comp) {
  orc_sim *s = (orc_sim *)h;
  s->filt_npass = npass;
  s->filt_comp = comp;
}

/* apply the current filter once (unit tests) */
void orc_filter_j(void *h) { filter_j((orc_sim *)h); }

static void field_half_b(orc_sim *s, double h) {
#pragma omp parallel for collapse(2) schedule(static)
  for (long k = 0; k < s->n[2]; ++k)
    for (long j = 0; j < s->n[1]; ++j)
      for (long i = 0; i < s->n[0]; ++i) {
        long id = i + s->n[0] * (j + s->n[1] * k);
        s->F[B1][id] -= h * (d2p(s, s->F[E3], i, j, k) - d3p(s, s->F[E2], i, j, k));
        s->F[B2][id] -= h * (d3p(s, s->F[E1], i, j, k) - d1p(s, s->F[E3], i, j, k));
        s->F[B3][id] -= h * (d1p(s, s->F[E2], i, j, k) - d2p(s, s->F[E1], i, j, k));
      }
}

static void field_e(orc_sim *s) {
  double dt = s->dt;
#pragma omp parallel for collapse(2) schedule(static)
  for (long k = 0; k < s->n[2]; ++k)
    for (long j = 0; j < s->n[1]; ++j)
      for (long i = 0; i < s->n[0]; ++i) {
        long id = i + s->n[0] * (j + s->n[1] * k);
        s->F[E1][id] += dt * (d2m(s, s->F[B3], i, j, k) - d3m(s, s->F[B2], i, j, k) - s->F[J1][id]);
        s->F[E2][id] += dt * (d3m(s, s->F[B1], i, j, k) - d1m(s, s->F[B3], i, j, k) - s->F[J2][id]);
        s->F[E3][id] += dt * (d1m(s, s->F[B2], i, j, k) - d2m(s, s->F[B1], i, j, k) - s->F[J3][id]);
      }
}

/* splitmix64 (Steele, Lea, Flood 2014): counter-based stream for the thermal
 * momenta of injected plasma; value k of stream `seed` is mix(seed + (k+1) G) */
static uint64_t smix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}
static double uni53(uint64_t seed, uint64_t k) {
  uint64_t z = smix(seed + (k + 1) * 0x9e3779b97f4a7c15ULL);
  return ((double)(z >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}
/* one normal deviate per index via Box-Muller on two uniforms */
static double normal_k(uint64_t seed, uint64_t k) {
  double a = uni53(seed, 2 * k), b = uni53(seed, 2 * k + 1);
  return sqrt(-2.0 * log(a)) * cos(2.0 * ORC_PI * b);
}

/* plasma injection at each window shift: ppc[d] particles per cell per
 * dimension on a regular sub-lattice, thermal momenta u_th * N(0,1) */
void orc_set_injection(void *h, const int *ppc, double Q, double qm, double uth, uint64_t seed) {
  orc_sim *s = (orc_sim *)h;
  s->inj_on = 1;
  for (int d = 0; d < 3; ++d) s->inj_ppc[d] = (d < s->ndim) ? ppc[d] : 1;
  s->inj_Q = Q;
  s->inj_qm = qm;
  s->inj_uth = uth;
  s->inj_seed = seed;
  s->inj_count = 0;
}

static void inject_slab(orc_sim *s, long i1g) {
  int *p = s->inj_ppc;
  long per = (long)p[0] * p[1] * p[2];
  long nnew = per * s->n[1] * s->n[2];
  grow(s, s->np + nnew);
  for (long k = 0; k < s->n[2]; ++k)
    for (long j = 0; j < s->n[1]; ++j)
      for (long q = 0; q < per; ++q) {
        long a = q % p[0], b = (q / p[0]) % p[1], c = q / (p[0] * p[1]);
        long id = s->np;
        double sub[3] = {(a + 0.5) / p[0] - 0.5, (b + 0.5) / p[1] - 0.5, (c + 0.5) / p[2] - 0.5};
        s->x[0][id] = (double)i1g + sub[0];
        s->x[1][id] = (double)j + sub[1];
        s->x[2][id] = (s->ndim == 3) ? (double)k + sub[2] : 0.0;
        for (int d = 0; d < 3; ++d)
          s->u[d][id] = s->inj_uth * normal_k(s->inj_seed, (uint64_t)(3 * s->inj_count + d));
        s->Q[id] = s->inj_Q;
        s->qm[id] = s->inj_qm;
        s->alive[id] = 1;
        s->inj_count++;
        s->np++;
      }
}

static void window_update(orc_sim *s) {
  if (!s->window) return;
  long target = (long)floor((double)s->step * s->vwin * s->dt / s->dx[0] + 1e-9);
  while (s->ws < target) {
    long n1 = s->n[0];
    for (int c = 0; c < 9; ++c) {
      for (long k = 0; k < s->n[2]; ++k)
        for (long j = 0; j < s->n[1]; ++j) {
          double *f = &s->F[c][n1 * (j + s->n[1] * k)];
          memmove(f, f + 1, sizeof(double) * (n1 - 1));
          f[n1 - 1] = 0.0;
        }
    }
    s->ws++;
    for (long p = 0; p < s->np; ++p) {
      if (!s->alive[p]) continue;
      long lg = (long)floor(s->x[0][p] + 0.5) - s->ws;
      if (lg < 2 || lg > n1 - 3) s->alive[p] = 0;
    }
    if (s->inj_on) inject_slab(s, s->ws + n1 - 3);
  }
}

void orc_step(void *h, long nsteps) {
  orc_sim *s = (orc_sim *)h;
  for (long it = 0; it < nsteps; ++it) {
    memset(s->F[J1], 0, sizeof(double) * s->N);
    memset(s->F[J2], 0, sizeof(double) * s->N);
    memset(s->F[J3], 0, sizeof(double) * s->N);
    long np = s->np;
    double *xn = (double *)malloc(sizeof(double) * 3 * (size_t)(np > 0 ? np : 1));
    double *un = (double *)malloc(sizeof(double) * 3 * (size_t)(np > 0 ? np : 1));
    /* gather at x^n, Boris push, new position: independent per particle */
#pragma omp parallel for schedule(dynamic, 256)
    for (long p = 0; p < np; ++p) {
      if (!s->alive[p]) continue;
      double xo[3] = {s->x[0][p], s->x[1][p], s->x[2][p]};
      double EB[6];
      gather(s, xo, EB);
      double u[3] = {s->u[0][p], s->u[1][p], s->u[2][p]};
      boris(s->qm[p], s->dt, EB, u);
      double g = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
      for (int d = 0; d < 3; ++d) {
        xn[3 * p + d] = (d < s->ndim) ? xo[d] + s->dt * u[d] / (g * s->dx[d]) : xo[d];
        un[3 * p + d] = u[d];
      }
    }
    /* current deposit in particle order (one shared J) */
    for (long p = 0; p < np; ++p) {
      if (!s->alive[p]) continue;
      double xo[3] = {s->x[0][p], s->x[1][p], s->x[2][p]};
      double *x1 = &xn[3 * p];
      double g = sqrt(1.0 + un[3 * p] * un[3 * p] + un[3 * p + 1] * un[3 * p + 1] + un[3 * p + 2] * un[3 * p + 2]);
      deposit(s, s->Q[p], xo, x1, un[3 * p + 2] / g);
      /* keep periodic coordinates in [-1/2, n - 1/2) */
      for (int d = 0; d < s->ndim; ++d) {
        if (d == 0 && s->window) continue;
        double nn = (double)s->n[d];
        if (x1[d] >= nn - 0.5) x1[d] -= nn;
        if (x1[d] < -0.5) x1[d] += nn;
      }
      for (int d = 0; d < 3; ++d) {
        s->x[d][p] = x1[d];
        s->u[d][p] = un[3 * p + d];
      }
    }
    free(xn);
    free(un);
    if (s->correct) correct_j1(s);
    if (s->filt_npass > 0) filter_j(s);
    field_half_b(s, 0.5 * s->dt);
    field_e(s);
    field_half_b(s, 0.5 * s->dt);
    s->step++;
    window_update(s);
  }
}

/* number of threads the parallel loops use (1 without OpenMP) */
int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ---- accessors -------------------------------------------------------- */
long orc_num_particles(void *h) { return ((orc_sim *)h)->np; }
long orc_window_start(void *h) { return ((orc_sim *)h)->ws; }
long orc_steps_done(void *h) { return ((orc_sim *)h)->step; }
long orc_correction_halfwidth(void *h) { return ((orc_sim *)h)->ng; }

void orc_get_field(void *h, int which, double *out) {
  orc_sim *s = (orc_sim *)h;
  memcpy(out, s->F[which], sizeof(double) * s->N);
}
void orc_set_field(void *h, int which, const double *in) {
  orc_sim *s = (orc_sim *)h;
  memcpy(s->F[which], in, sizeof(double) * s->N);
}
/* x: [np][3], u: [np][3], alive: [np] */
void orc_get_particles(void *h, double *x, double *u, int *alive) {
  orc_sim *s = (orc_sim *)h;
  for (long p = 0; p < s->np; ++p) {
    for (int d = 0; d < 3; ++d) {
      x[3 * p + d] = s->x[d][p];
      u[3 * p + d] = s->u[d][p];
    }
    alive[p] = s->alive[p];
  }
}

/* node charge density of the alive particles at their current positions */
void orc_rho(void *h, double *out) {
  orc_sim *s = (orc_sim *)h;
  memset(out, 0, sizeof(double) * s->N);
  double dV = s->dx[0] * s->dx[1] * (s->ndim == 3 ? s->dx[2] : 1.0);
  for (long p = 0; p < s->np; ++p) {
    if (!s->alive[p]) continue;
    long c[3] = {0, 0, 0};
    for (int d = 0; d < s->ndim; ++d) c[d] = (long)floor(s->x[d][p] + 0.5);
    long kr = (s->ndim == 3) ? 2 : 0;
    for (long k = c[2] - kr; k <= c[2] + kr; ++k) {
      double w3 = (s->ndim == 3) ? spline2((double)k - s->x[2][p]) : 1.0;
      for (long j = c[1] - 2; j <= c[1] + 2; ++j) {
        double w2 = spline2((double)j - s->x[1][p]);
        for (long i = c[0] - 2; i <= c[0] + 2; ++i) {
          double w1 = spline2((double)i - s->x[0][p]);
          double w = w1 * w2 * w3;
          if (w == 0.0) continue;
          double *r = fref(s, out, i - s->ws, j, k);
          if (r) *r += s->Q[p] * w / dV;
        }
      }
    }
  }
}

/* discrete divergence d- . E at the nodes (customized operator along x1) */
void orc_div_e(void *h, double *out) {
  orc_sim *s = (orc_sim *)h;
  for (long k = 0; k < s->n[2]; ++k)
    for (long j = 0; j < s->n[1]; ++j)
      for (long i = 0; i < s->n[0]; ++i) {
        long id = i + s->n[0] * (j + s->n[1] * k);
        out[id] = d1m(s, s->F[E1], i, j, k) + d2m(s, s->F[E2], i, j, k) + d3m(s, s->F[E3], i, j, k);
      }
}

/* field energy 1/2 sum (E^2 + B^2) dV and kinetic energy sum m_macro (gamma-1) */
void orc_energy(void *h, double *wf, double *wk) {
  orc_sim *s = (orc_sim *)h;
  double dV = s->dx[0] * s->dx[1] * (s->ndim == 3 ? s->dx[2] : 1.0);
  double acc = 0.0;
  for (int c = 0; c < 6; ++c)
    for (long i = 0; i < s->N; ++i) acc += s->F[c][i] * s->F[c][i];
  *wf = 0.5 * acc * dV;
  double kin = 0.0;
  for (long p = 0; p < s->np; ++p) {
    if (!s->alive[p]) continue;
    double g = sqrt(1.0 + s->u[0][p] * s->u[0][p] + s->u[1][p] * s->u[1][p] + s->u[2][p] * s->u[2][p]);
    kin += (s->Q[p] / s->qm[p]) * (g - 1.0);
  }
  *wk = kin;
}

/* apply only the field advance (steps 6 of the cycle) with J held at zero:
 * used by the vacuum dispersion tests */
void orc_field_only(void *h, long nsteps) {
  orc_sim *s = (orc_sim *)h;
  for (long it = 0; it < nsteps; ++it) {
    memset(s->F[J1], 0, sizeof(double) * s->N);
    memset(s->F[J2], 0, sizeof(double) * s->N);
    memset(s->F[J3], 0, sizeof(double) * s->N);
    field_half_b(s, 0.5 * s->dt);
    field_e(s);
    field_half_b(s, 0.5 * s->dt);
    s->step++;
  }
}

/* Boris push of standalone particles in given fields (unit tests) */
void orc_boris(double qm, double dt, const double *EB, double *u) { boris(qm, dt, EB, u); }

/* Esirkepov current of one particle moving xo -> xn written into J (3 arrays
 * of the grid), with the grid otherwise untouched: unit tests of continuity */
void orc_deposit_one(void *h, double Q, const double *xo, const double *xn, double v3) {
  orc_sim *s = (orc_sim *)h;
  double a[3] = {0, 0, 0}, b[3] = {0, 0, 0};
  for (int d = 0; d < s->ndim; ++d) {
    a[d] = xo[d];
    b[d] = xn[d];
  }
  deposit(s, Q, a, b, v3);
}

/* apply the J1 correction once to the current J1 array (unit tests) */
void orc_correct_j1(void *h) { correct_j1((orc_sim *)h); }
