/*
 * FP64 CPU oracle for periodic cubic-spline particle tracking.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain, obviously-correct
 * statement of what the GPU path computes.  Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it.  It shares no code,
 * header, constant or table with the GPU library: every formula below is
 * written out again from the paper (Buaria & Yeung, "A highly scalable
 * particle tracking algorithm using partitioned global address space (PGAS)
 * programming for extreme-scale turbulence simulations") and from the
 * mathematics of periodic cubic splines.
 *
 * Conventions (all arrays in host memory, x the fastest index):
 *   field  [3][nz][ny][nx]              grid values g of (u,v,w), FP64
 *   coeff  [3][nz+3][ny+3][nx+3]        padded spline coefficients S, FP64;
 *                                       padded index P holds S[(P-1) mod n]
 *   pos    [3][np]                      particle positions (x, y, z), FP64,
 *                                       unwrapped (any real value)
 *   out    [3][np] or [12][np]          u,v,w then du_i/dx_j (i outer)
 *
 * Readings of the paper taken here (the paper is silent or ambiguous):
 *   - basis functions: uniform cubic B-spline pieces normalised to a
 *     partition of unity (Sec. 2.2 defers their form to Yeung & Pope 1988;
 *     the interpolant does not depend on the scaling);
 *   - the periodic tridiagonal system is solved by Thomas elimination with a
 *     Sherman-Morrison rank-one correction for the two corner entries;
 *   - cell membership is half-open, alpha = floor(x/dx) of the shadow
 *     position;
 *   - the particle RK2 scheme is Heun's predictor-corrector;
 *   - inertial particles (Sec. 4.3 names them without an equation) follow
 *     Stokes drag, advanced by the exponential-integrator form of Heun's
 *     step given at oracle_inertial_step.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_ERR_SIZE (-2)
#define OR_ERR_NONFINITE (-5)

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of the parallel loops that follow (timing on one core). */
void oracle_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Operation 1: spline coefficients (Sec. 2.2).                              */
/* ------------------------------------------------------------------------ */

/* Plain Thomas elimination for a tridiagonal system with constant sub- and
 * super-diagonal entries (lo, up) and diagonal diag[0..n-1]. */
static void thomas(int n, const double *diag, double lo, double up,
                   const double *rhs, double *x, double *cp, double *dp) {
  cp[0] = up / diag[0];
  dp[0] = rhs[0] / diag[0];
  for (int i = 1; i < n; ++i) {
    double den = diag[i] - lo * cp[i - 1];
    cp[i] = up / den;
    dp[i] = (rhs[i] - lo * dp[i - 1]) / den;
  }
  x[n - 1] = dp[n - 1];
  for (int i = n - 2; i >= 0; --i) x[i] = dp[i] - cp[i] * x[i + 1];
}

/* Solve (S[m-1] + 4 S[m] + S[m+1]) / 6 = g[m], m = 0..n-1, indices mod n:
 * the periodic tridiagonal system of one grid line (Sec. 2.2, "tridiagonal
 * system ... with periodicity in space", solved by the Thomas algorithm).
 * The cyclic matrix A is split as A = T + u v^T with T tridiagonal:
 *   u = (gam, 0, .., 0, beta)^T,  v = (1, 0, .., 0, alpha/gam)^T,
 * alpha = A[0][n-1], beta = A[n-1][0], gam = -A[0][0].  Then
 *   S = y - (v.y)/(1 + v.z) z,  T y = g,  T z = u  (Sherman-Morrison).
 * Requires n >= 3.  `work` holds 6n doubles. */
static void solve_periodic_line(int n, const double *g, double *S,
                                double *work) {
  const double dg = 4.0 / 6.0, off = 1.0 / 6.0;
  const double alpha = off, beta = off, gam = -dg;
  double *diag = work, *y = work + n, *z = work + 2 * n, *u = work + 3 * n;
  double *cp = work + 4 * n, *dp = work + 5 * n;
  for (int i = 0; i < n; ++i) { diag[i] = dg; u[i] = 0.0; }
  diag[0] = dg - gam;
  diag[n - 1] = dg - alpha * beta / gam;
  u[0] = gam;
  u[n - 1] = beta;
  thomas(n, diag, off, off, g, y, cp, dp);
  thomas(n, diag, off, off, u, z, cp, dp);
  double vy = y[0] + (alpha / gam) * y[n - 1];
  double vz = z[0] + (alpha / gam) * z[n - 1];
  double f = vy / (1.0 + vz);
  for (int i = 0; i < n; ++i) S[i] = y[i] - f * z[i];
}

/* Public 1-D entry (used by the tests that pin the solve). */
int oracle_solve_line(int n, const double *g, double *S) {
  if (n < 3) return OR_ERR_SIZE;
  double *work = (double *)malloc(sizeof(double) * 6 * (size_t)n);
  solve_periodic_line(n, g, S, work);
  free(work);
  return OR_OK;
}

/* Apply the periodic line solve along one axis of an n0 x n1 x n2 array
 * (n2 fastest), in place.  axis = 0 (slowest, z), 1 (y) or 2 (x). */
static void solve_axis(int nz, int ny, int nx, double *a, int axis) {
  int len = axis == 2 ? nx : axis == 1 ? ny : nz;
  int64_t stride = axis == 2 ? 1 : axis == 1 ? nx : (int64_t)nx * ny;
  int64_t nlines = ((int64_t)nx * ny * nz) / len;
#pragma omp parallel
  {
    double *g = (double *)malloc(sizeof(double) * len);
    double *s = (double *)malloc(sizeof(double) * len);
    double *work = (double *)malloc(sizeof(double) * 6 * (size_t)len);
#pragma omp for schedule(static)
    for (int64_t l = 0; l < nlines; ++l) {
      int64_t base;
      if (axis == 2) {
        base = l * nx;
      } else if (axis == 1) {
        int64_t zi = l / nx, xi = l % nx;
        base = zi * (int64_t)nx * ny + xi;
      } else {
        base = l; /* (y, x) plane index */
      }
      for (int m = 0; m < len; ++m) g[m] = a[base + m * stride];
      solve_periodic_line(len, g, s, work);
      for (int m = 0; m < len; ++m) a[base + m * stride] = s[m];
    }
    free(g);
    free(s);
    free(work);
  }
}

static inline int wrapi(int i, int n) { return ((i % n) + n) % n; }

/* Spline coefficients of (u,v,w) (Operation 1 of Sec. 2.2): per component,
 * the periodic solve along x, then z, then y (the paper's order), followed by
 * the padding to (n+3) coefficients per line (index range 1..N+3 of
 * eq. (spline)): padded index P holds S[(P-1) mod n] along every axis. */
int oracle_spline_coeffs(int nx, int ny, int nz, const double *field,
                         double *coeff) {
  if (nx < 4 || ny < 4 || nz < 4) return OR_ERR_SIZE;
  int64_t npts = (int64_t)nx * ny * nz;
  int px = nx + 3, py = ny + 3, pz = nz + 3;
  int64_t ppts = (int64_t)px * py * pz;
  double *a = (double *)malloc(sizeof(double) * npts);
  for (int c = 0; c < 3; ++c) {
    memcpy(a, field + c * npts, sizeof(double) * npts);
    solve_axis(nz, ny, nx, a, 2); /* x */
    solve_axis(nz, ny, nx, a, 0); /* z */
    solve_axis(nz, ny, nx, a, 1); /* y */
    double *o = coeff + c * ppts;
#pragma omp parallel for schedule(static)
    for (int Z = 0; Z < pz; ++Z)
      for (int Y = 0; Y < py; ++Y)
        for (int X = 0; X < px; ++X) {
          int zi = wrapi(Z - 1, nz), yi = wrapi(Y - 1, ny), xi = wrapi(X - 1, nx);
          o[((int64_t)Z * py + Y) * px + X] = a[((int64_t)zi * ny + yi) * nx + xi];
        }
  }
  free(a);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Position -> cell, local coordinate and sort key (Sec. 2.2 and Sec. 3).    */
/* ------------------------------------------------------------------------ */

/* Shadow position and cell along one axis.  A position outside [0, L) is
 * shifted by a multiple of L (Sec. 2.2, periodic "shadow" location; Sec. 3,
 * modulo mapping).  In grid units s = x * (n / L):
 *   s_w = s - n floor(s / n), corrected once into [0, n);
 *   alpha = floor(s_w) in [0, n-1];  t = s_w - alpha in [0, 1).
 * Every operation is a single IEEE-754 double operation, none contracted. */
static void cell_1d(double x, double cscale, int n, int *alpha, double *t) {
  double dn = (double)n;
  double s = x * cscale;
  double k = floor(s / dn);
  double kn = k * dn;
  double sw = s - kn;
  if (sw < 0.0) sw = sw + dn;
  if (sw >= dn) sw = sw - dn;
  double fa = floor(sw);
  *alpha = (int)fa;
  *t = sw - fa;
}

/* Sort key of a cell (alpha, beta, gamma): cells are grouped into columns of
 * tx * ty cells in the (x, y) plane that run the full height in z; the key
 * orders particles by column, then z, then y, then x inside the column:
 *   key = (((cy * ncx + cx) * nz + gamma) * ty + ly) * tx + lx,
 * cx = alpha / tx, lx = alpha % tx, cy = beta / ty, ly = beta % ty,
 * ncx = ceil(nx / tx).  (The paper assigns each particle to the process that
 * owns its sub-domain, Sec. 3; on one device the analogue is ordering the
 * particles by the cell that holds them.) */
static uint64_t cell_key(int a, int b, int g, int nx, int nz, int tx, int ty) {
  uint64_t ncx = (uint64_t)((nx + tx - 1) / tx);
  uint64_t cx = (uint64_t)(a / tx), lx = (uint64_t)(a % tx);
  uint64_t cy = (uint64_t)(b / ty), ly = (uint64_t)(b % ty);
  return (((cy * ncx + cx) * (uint64_t)nz + (uint64_t)g) * (uint64_t)ty + ly) *
             (uint64_t)tx + lx;
}

/* cells [3][np] (int32, may be NULL), t [3][np] (may be NULL),
 * key [np] (may be NULL).  Returns OR_ERR_NONFINITE if any coordinate is
 * NaN or infinite (outputs for such particles are left unspecified). */
int oracle_cell_keys(int nx, int ny, int nz, double lx, double ly, double lz,
                     int tx, int ty, int64_t np, const double *pos,
                     int32_t *cells, double *t, uint64_t *key) {
  double cs[3] = {(double)nx / lx, (double)ny / ly, (double)nz / lz};
  int n[3] = {nx, ny, nz};
  int bad = 0;
  for (int64_t p = 0; p < np; ++p) {
    int ab[3];
    double tt[3];
    for (int d = 0; d < 3; ++d) {
      double x = pos[d * np + p];
      if (!isfinite(x)) { bad = 1; ab[d] = 0; tt[d] = 0.0; continue; }
      cell_1d(x, cs[d], n[d], &ab[d], &tt[d]);
    }
    for (int d = 0; d < 3; ++d) {
      if (cells) cells[d * np + p] = ab[d];
      if (t) t[d * np + p] = tt[d];
    }
    if (key) key[p] = cell_key(ab[0], ab[1], ab[2], nx, nz, tx, ty);
  }
  return bad ? OR_ERR_NONFINITE : OR_OK;
}

/* Stable sort of particle indices by key: perm[i] is the original index of
 * the particle placed at sorted position i; equal keys keep input order.
 * Plain top-down merge sort. */
static void merge_sort(int32_t *a, int32_t *tmp, int64_t lo, int64_t hi,
                       const uint64_t *key) {
  if (hi - lo < 2) return;
  int64_t mid = lo + (hi - lo) / 2;
  merge_sort(a, tmp, lo, mid, key);
  merge_sort(a, tmp, mid, hi, key);
  int64_t i = lo, j = mid, o = lo;
  while (i < mid && j < hi) {
    if (key[a[j]] < key[a[i]]) tmp[o++] = a[j++];
    else tmp[o++] = a[i++];
  }
  while (i < mid) tmp[o++] = a[i++];
  while (j < hi) tmp[o++] = a[j++];
  for (int64_t q = lo; q < hi; ++q) a[q] = tmp[q];
}

void oracle_stable_sort(int64_t np, const uint64_t *key, int32_t *perm) {
  int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * (np > 0 ? np : 1));
  for (int64_t i = 0; i < np; ++i) perm[i] = (int32_t)i;
  merge_sort(perm, tmp, 0, np, key);
  free(tmp);
}

/* ------------------------------------------------------------------------ */
/* Operations 2 and 3: basis functions and the 64-term sum (eq. (spline)).  */
/* ------------------------------------------------------------------------ */

/* The four 1-D basis functions at local coordinate t in [0,1): the pieces of
 * the uniform cubic B-spline that overlap the cell, ordered i = 1..4 for the
 * coefficients at p = alpha-1 .. alpha+2 (eq. (spline), p = alpha + i - 2).
 * They have compact support over four grid spacings (Sec. 2.2). */
static void basis(double t, double w[4]) {
  double s = 1.0 - t;
  w[0] = s * s * s / 6.0;
  w[1] = (3.0 * t * t * t - 6.0 * t * t + 4.0) / 6.0;
  w[2] = (-3.0 * t * t * t + 3.0 * t * t + 3.0 * t + 1.0) / 6.0;
  w[3] = t * t * t / 6.0;
}

/* d/dt of the four basis functions. */
static void basis_dt(double t, double w[4]) {
  double s = 1.0 - t;
  w[0] = -s * s / 2.0;
  w[1] = (9.0 * t * t - 12.0 * t) / 6.0;
  w[2] = (-9.0 * t * t + 6.0 * t + 3.0) / 6.0;
  w[3] = t * t / 2.0;
}

typedef struct {
  int nx, ny, nz;
  double lx, ly, lz;
} or_grid;

/* Per-particle evaluation.  out12[0..2] = (u,v,w); when want_grad,
 * out12[3 + 3c + d] = d u_c / d x_d (physical units). */
static void eval_particle(const or_grid *gr, const double *coeff, double x,
                          double y, double z, int want_grad, double *out12) {
  int n[3] = {gr->nx, gr->ny, gr->nz};
  double L[3] = {gr->lx, gr->ly, gr->lz};
  double xyz[3] = {x, y, z};
  int a[3];
  double t[3], w[3][4], dw[3][4];
  for (int d = 0; d < 3; ++d) {
    cell_1d(xyz[d], (double)n[d] / L[d], n[d], &a[d], &t[d]);
    basis(t[d], w[d]);
    basis_dt(t[d], dw[d]);
    double inv_h = (double)n[d] / L[d];
    for (int i = 0; i < 4; ++i) dw[d][i] *= inv_h;
  }
  int px = gr->nx + 3, py = gr->ny + 3, pz = gr->nz + 3;
  int64_t ppts = (int64_t)px * py * pz;
  for (int q = 0; q < 12; ++q) out12[q] = 0.0;
  for (int c = 0; c < 3; ++c) {
    const double *S = coeff + c * ppts;
    double v = 0, gx = 0, gy = 0, gz = 0;
    for (int k = 0; k < 4; ++k)
      for (int j = 0; j < 4; ++j)
        for (int i = 0; i < 4; ++i) {
          /* padded index = (alpha + i - 2) + 1 with i = 1..4 */
          int64_t idx = ((int64_t)(a[2] + k) * py + (a[1] + j)) * px + (a[0] + i);
          double s = S[idx];
          v += w[0][i] * w[1][j] * w[2][k] * s;
          if (want_grad) {
            gx += dw[0][i] * w[1][j] * w[2][k] * s;
            gy += w[0][i] * dw[1][j] * w[2][k] * s;
            gz += w[0][i] * w[1][j] * dw[2][k] * s;
          }
        }
    out12[c] = v;
    if (want_grad) {
      out12[3 + 3 * c + 0] = gx;
      out12[3 + 3 * c + 1] = gy;
      out12[3 + 3 * c + 2] = gz;
    }
  }
}

static int check_finite(int64_t np, const double *pos) {
  for (int64_t i = 0; i < 3 * np; ++i)
    if (!isfinite(pos[i])) return 0;
  return 1;
}

/* Interpolated (u,v,w) (n_out = 3) or (u,v,w) plus the nine velocity
 * gradients (n_out = 12) at every particle; out is [n_out][np]. */
int oracle_interp(int nx, int ny, int nz, double lx, double ly, double lz,
                  const double *coeff, int64_t np, const double *pos,
                  int n_out, double *out) {
  if (n_out != 3 && n_out != 12) return OR_ERR_SIZE;
  if (!check_finite(np, pos)) return OR_ERR_NONFINITE;
  or_grid gr = {nx, ny, nz, lx, ly, lz};
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < np; ++p) {
    double o[12];
    eval_particle(&gr, coeff, pos[p], pos[np + p], pos[2 * np + p], n_out == 12, o);
    for (int q = 0; q < n_out; ++q) out[q * np + p] = o[q];
  }
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Particle advance: dx+/dt = u(x+, t) (eq. (dxdt)), one explicit RK2 step   */
/* per call, Heun's form: u0 = u(x), x* = x + dt u0, u1 = u(x*),             */
/* x <- x + dt/2 (u0 + u1).  Positions stay unwrapped.                      */
/* ------------------------------------------------------------------------ */
int oracle_rk2_step(int nx, int ny, int nz, double lx, double ly, double lz,
                    const double *coeff, int64_t np, double dt, double *pos) {
  if (!check_finite(np, pos)) return OR_ERR_NONFINITE;
  or_grid gr = {nx, ny, nz, lx, ly, lz};
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < np; ++p) {
    double x0[3] = {pos[p], pos[np + p], pos[2 * np + p]};
    double u0[12], u1[12], xs[3];
    eval_particle(&gr, coeff, x0[0], x0[1], x0[2], 0, u0);
    for (int d = 0; d < 3; ++d) xs[d] = x0[d] + dt * u0[d];
    eval_particle(&gr, coeff, xs[0], xs[1], xs[2], 0, u1);
    for (int d = 0; d < 3; ++d) pos[d * np + p] = x0[d] + 0.5 * dt * (u0[d] + u1[d]);
  }
  return OR_OK;
}

/* One Heun step in a field that changes over the step.  In the paper's
 * production runs (Sec. 4.3, Table 5) the particles are advanced at each
 * sub-step of the flow solver's second-order Runge-Kutta scheme, with spline
 * coefficients recomputed from the velocity field of that sub-step: the
 * predictor uses the field at t_n, the corrector the field at t_n + dt.
 *   u0 = u^n(x);  x* = x + dt u0;  x <- x + dt/2 (u0 + u^{n+1}(x*)). */
/* phi_m(r) = sum_{j>=0} (-r)^j / (j+m)!, the functions of exponential
 * integrators: phi_1 = (1 - e^-r)/r, phi_2 = (1 - phi_1)/r,
 * phi_3 = (1/2 - phi_2)/r.  The recursions lose digits to cancellation for
 * small r, so there the series is summed (15 terms: truncation below 1e-27). */
static void phi123(double r, double *p1, double *p2, double *p3) {
  if (r >= 0.1) {
    *p1 = (1.0 - exp(-r)) / r;
    *p2 = (1.0 - *p1) / r;
    *p3 = (0.5 - *p2) / r;
    return;
  }
  double s[3] = {0.0, 0.0, 0.0};
  for (int m = 1; m <= 3; ++m) {
    double fact = 1.0; /* m! */
    for (int q = 2; q <= m; ++q) fact *= q;
    double term = 1.0 / fact, sum = 0.0;
    for (int j = 0; j < 15; ++j) {
      sum += term;
      term *= -r / (double)(j + 1 + m);
    }
    s[m - 1] = sum;
  }
  *p1 = s[0];
  *p2 = s[1];
  *p3 = s[2];
}

/* Inertial (or diffusive) particle step: Sec. 4.3 notes that inertial
 * particles, or markers with a high molecular diffusivity, can move more than
 * one grid spacing per step.  The paper gives no equation for them; reading
 * taken here: the Stokes-drag particle
 *   dx/dt = v,   dv/dt = (u(x) - v) / tau,
 * advanced over a step h by the exact solution of these equations with the
 * fluid velocity seen along the step taken as linear in time, from
 * u0 = u(x^n) to u1 = u(x*) at the predicted end point x* (the position the
 * exact solution reaches if the fluid velocity stays u0), i.e. an
 * exponential-integrator form of Heun's predictor-corrector.  With
 * r = h/tau, E = exp(-r):
 *   x*   = x + h phi_1 v + h r phi_2 u0 + d
 *   x+   = x* + h r phi_3 (u1 - u0)
 *   v+   = E v + (phi_1 - E) u0 + r phi_2 u1,
 * (written out: h phi_1 = tau (1 - E), h r phi_2 = h - tau (1 - E),
 * h r phi_3 = h/2 - tau + tau^2 (1 - E)/h), where d is an optional
 * displacement increment per particle (the random displacement
 * sqrt(2 kappa h) xi of a diffusive marker, drawn by the caller), added to
 * the predictor and kept in the corrector.  tau = 0 is the fluid tracer: the
 * limits phi_1 -> 0, r phi_2 -> 1, r phi_3 -> 1/2, E -> 0 give Heun's step
 * x+ = x + h/2 (u0 + u1) + d with v+ = u1.  vel may be NULL only when tau = 0
 * (then not read or written). */
int oracle_inertial_step(int nx, int ny, int nz, double lx, double ly, double lz,
                         const double *coeff, int64_t np, double dt, double tau,
                         double *pos, double *vel, const double *disp) {
  if (!check_finite(np, pos)) return OR_ERR_NONFINITE;
  if (!(tau >= 0.0) || !(dt > 0.0) || (tau > 0.0 && !vel)) return OR_ERR_SIZE;
  or_grid gr = {nx, ny, nz, lx, ly, lz};
  double E = 0.0, cv = 0.0, cu = dt, c1 = 0.5 * dt, b = 1.0;
  if (tau > 0.0) {
    const double r = dt / tau;
    double p1, p2, p3;
    phi123(r, &p1, &p2, &p3);
    E = exp(-r);
    cv = dt * p1;      /* coefficient of v in the predictor */
    cu = dt * r * p2;  /* of u0 in the predictor */
    c1 = dt * r * p3;  /* of (u1 - u0) in the corrector */
    b = r * p2;        /* of u1 in the new velocity */
  }
  const double bu0 = tau > 0.0 ? (cv / dt - E) : 0.0; /* of u0 in the new velocity */
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < np; ++p) {
    double x0[3], v0[3], dd[3], xs[3], u0[12], u1[12];
    for (int d = 0; d < 3; ++d) {
      x0[d] = pos[d * np + p];
      v0[d] = tau > 0.0 ? vel[d * np + p] : 0.0;
      dd[d] = disp ? disp[d * np + p] : 0.0;
    }
    eval_particle(&gr, coeff, x0[0], x0[1], x0[2], 0, u0);
    for (int d = 0; d < 3; ++d) xs[d] = x0[d] + cv * v0[d] + cu * u0[d] + dd[d];
    eval_particle(&gr, coeff, xs[0], xs[1], xs[2], 0, u1);
    for (int d = 0; d < 3; ++d) {
      pos[d * np + p] = xs[d] + c1 * (u1[d] - u0[d]);
      if (vel) vel[d * np + p] = E * v0[d] + bu0 * u0[d] + b * u1[d];
    }
  }
  return OR_OK;
}

int oracle_rk2_step_tv(int nx, int ny, int nz, double lx, double ly, double lz,
                       const double *coeff_n, const double *coeff_np1, int64_t np,
                       double dt, double *pos) {
  if (!check_finite(np, pos)) return OR_ERR_NONFINITE;
  or_grid gr = {nx, ny, nz, lx, ly, lz};
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < np; ++p) {
    double x0[3] = {pos[p], pos[np + p], pos[2 * np + p]};
    double u0[12], u1[12], xs[3];
    eval_particle(&gr, coeff_n, x0[0], x0[1], x0[2], 0, u0);
    for (int d = 0; d < 3; ++d) xs[d] = x0[d] + dt * u0[d];
    eval_particle(&gr, coeff_np1, xs[0], xs[1], xs[2], 0, u1);
    for (int d = 0; d < 3; ++d) pos[d * np + p] = x0[d] + 0.5 * dt * (u0[d] + u1[d]);
  }
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Adjoints (hand-derived; the paper has no differentiation).               */
/* ------------------------------------------------------------------------ */

/* Scatter of one particle's weights times gu[3] into g_coeff (transposed
 * 64-term sum), and the position adjoint gpos[d] += sum_c gu[c] du_c/dx_d. */
static void particle_bwd(const or_grid *gr, const double *coeff, const double xyz[3],
                         const double gu[3], double gpos[3], double *gcoeff) {
  int n[3] = {gr->nx, gr->ny, gr->nz};
  double L[3] = {gr->lx, gr->ly, gr->lz};
  int a[3];
  double t[3], w[3][4];
  for (int d = 0; d < 3; ++d) {
    cell_1d(xyz[d], (double)n[d] / L[d], n[d], &a[d], &t[d]);
    basis(t[d], w[d]);
  }
  double o[12];
  eval_particle(gr, coeff, xyz[0], xyz[1], xyz[2], 1, o);
  for (int d = 0; d < 3; ++d)
    for (int c = 0; c < 3; ++c) gpos[d] += gu[c] * o[3 + 3 * c + d];
  if (!gcoeff) return;
  int px = gr->nx + 3, py = gr->ny + 3, pz = gr->nz + 3;
  int64_t ppts = (int64_t)px * py * pz;
  for (int k = 0; k < 4; ++k)
    for (int j = 0; j < 4; ++j)
      for (int i = 0; i < 4; ++i) {
        int64_t idx = ((int64_t)(a[2] + k) * py + (a[1] + j)) * px + (a[0] + i);
        double wt = w[0][i] * w[1][j] * w[2][k];
        for (int c = 0; c < 3; ++c) gcoeff[c * ppts + idx] += wt * gu[c];
      }
}

/* Adjoint of oracle_interp with n_out = 3: given gout = dL/d(u,v,w) [3][np],
 * accumulate gpos += (du/dx)^T gout and gcoeff += W^T gout (either may be
 * NULL).  Serial, so the accumulation order is fixed. */
int oracle_interp_bwd(int nx, int ny, int nz, double lx, double ly, double lz,
                      const double *coeff, int64_t np, const double *pos,
                      const double *gout, double *gpos, double *gcoeff) {
  if (!check_finite(np, pos)) return OR_ERR_NONFINITE;
  or_grid gr = {nx, ny, nz, lx, ly, lz};
  for (int64_t p = 0; p < np; ++p) {
    double xyz[3] = {pos[p], pos[np + p], pos[2 * np + p]};
    double gu[3] = {gout[p], gout[np + p], gout[2 * np + p]};
    double gp[3] = {0, 0, 0};
    particle_bwd(&gr, coeff, xyz, gu, gp, gcoeff);
    if (gpos)
      for (int d = 0; d < 3; ++d) gpos[d * np + p] += gp[d];
  }
  return OR_OK;
}

/* Adjoint of oracle_spline_coeffs: fold the padded layers back onto the n
 * grid points they copy (g[(P-1) mod n] += gpad[P] along every axis), then
 * apply the transposed line solves.  The 1-4-1 cyclic matrix is symmetric, so
 * each transposed solve is the same periodic solve; they are applied in the
 * reverse of the forward order (y, z, x).  gfield is overwritten. */
int oracle_spline_coeffs_bwd(int nx, int ny, int nz, const double *gcoeff,
                             double *gfield) {
  if (nx < 4 || ny < 4 || nz < 4) return OR_ERR_SIZE;
  int64_t npts = (int64_t)nx * ny * nz;
  int px = nx + 3, py = ny + 3, pz = nz + 3;
  int64_t ppts = (int64_t)px * py * pz;
  for (int c = 0; c < 3; ++c) {
    double *a = gfield + c * npts;
    const double *gp = gcoeff + c * ppts;
    memset(a, 0, sizeof(double) * npts);
    for (int Z = 0; Z < pz; ++Z)
      for (int Y = 0; Y < py; ++Y)
        for (int X = 0; X < px; ++X) {
          int zi = wrapi(Z - 1, nz), yi = wrapi(Y - 1, ny), xi = wrapi(X - 1, nx);
          a[((int64_t)zi * ny + yi) * nx + xi] += gp[((int64_t)Z * py + Y) * px + X];
        }
    solve_axis(nz, ny, nx, a, 1); /* y */
    solve_axis(nz, ny, nx, a, 0); /* z */
    solve_axis(nz, ny, nx, a, 2); /* x */
  }
  return OR_OK;
}

/* Adjoint of one Heun step.  pos_n are the positions the step started from;
 * on entry gpos = lambda = dL/dx^{n+1}, on exit gpos = dL/dx^n.  With
 * J(x) = du/dx and W(x) the 64-term weights:
 *   ub1 = ub0 = dt/2 lambda;  xbs = J(x*)^T ub1;  ub0 += dt xbs;
 *   xbn = lambda + xbs + J(x^n)^T ub0;
 *   gcoeff += W(x*)^T ub1 + W(x^n)^T ub0  (gcoeff may be NULL). */
/* Particles are independent: large particle sets are split into contiguous
 * blocks, one per thread, each summing its W^T terms into a private copy of
 * gcoeff; the copies are then added in block order (only the rounding of
 * the FP64 sums depends on the thread count). */
int oracle_rk2_step_bwd(int nx, int ny, int nz, double lx, double ly, double lz,
                        const double *coeff, int64_t np, double dt,
                        const double *pos_n, double *gpos, double *gcoeff) {
  if (!check_finite(np, pos_n)) return OR_ERR_NONFINITE;
  or_grid gr = {nx, ny, nz, lx, ly, lz};
  const int64_t ppts = 3 * (int64_t)(nx + 3) * (ny + 3) * (nz + 3);
  int nt = oracle_num_threads();
  if (np < 4096 || nt < 2) nt = 1;
  double *priv = NULL;
  if (nt > 1 && gcoeff) {
    priv = (double *)calloc((size_t)nt * ppts, sizeof(double));
    if (!priv) nt = 1;
  }
#pragma omp parallel for schedule(static, 1) num_threads(nt) if (nt > 1)
  for (int b = 0; b < nt; ++b) {
    const int64_t p0 = np * b / nt, p1 = np * (b + 1) / nt;
    double *gc = gcoeff ? (priv ? priv + (int64_t)b * ppts : gcoeff) : NULL;
    for (int64_t p = p0; p < p1; ++p) {
      double x0[3] = {pos_n[p], pos_n[np + p], pos_n[2 * np + p]};
      double u0[12], xs[3];
      eval_particle(&gr, coeff, x0[0], x0[1], x0[2], 0, u0);
      for (int d = 0; d < 3; ++d) xs[d] = x0[d] + dt * u0[d];
      double lam[3] = {gpos[p], gpos[np + p], gpos[2 * np + p]};
      double ub1[3], ub0[3], xbs[3] = {0, 0, 0}, xbn[3] = {0, 0, 0};
      for (int d = 0; d < 3; ++d) ub1[d] = ub0[d] = 0.5 * dt * lam[d];
      particle_bwd(&gr, coeff, xs, ub1, xbs, gc);
      for (int d = 0; d < 3; ++d) ub0[d] += dt * xbs[d];
      particle_bwd(&gr, coeff, x0, ub0, xbn, gc);
      for (int d = 0; d < 3; ++d) gpos[d * np + p] = lam[d] + xbs[d] + xbn[d];
    }
  }
  if (priv) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < ppts; ++i) {
      double s = gcoeff[i];
      for (int b = 0; b < nt; ++b) s += priv[(int64_t)b * ppts + i];
      gcoeff[i] = s;
    }
    free(priv);
  }
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Coefficients from the closed-form periodic inverse, at chosen points.     */
/* ------------------------------------------------------------------------ */
/* The inverse of the periodic system (S[m-1] + 4 S[m] + S[m+1]) / 6 = g[m]  */
/* of Operation 1 has the closed form                                        */
/*   (A^-1)[m][m'] = sqrt(3) (z^d + z^(n-d)) / (1 - z^n),                     */
/*   d = (m - m') mod n,  z = sqrt(3) - 2,                                    */
/* so S at one grid point is a weighted sum of the line's g values whose      */
/* weights decay like |z|^d (|z| = 0.268).  Summing d over [-W, W] instead   */
/* of the whole line leaves out at most 2 sqrt(3) |z|^(W+1) / (1 - |z|)      */
/* times max |g| (4.6e-16 max |g| for W = 28); lines with n <= 2 W + 1 are   */
/* summed in full.  The 3-D coefficients are the product of the three line   */
/* inverses (tensor-product interpolant), applied axis by axis over the      */
/* window around the 4 x 4 x 4 stencil of each particle.  This restates      */
/* Operation 1 through a different exact method than the Thomas solve above, */
/* for grids too large for a full FP64 solve on the host.                    */

static double inv_entry(int n, int d) {
  const double z = sqrt(3.0) - 2.0;
  d = wrapi(d, n);
  return sqrt(3.0) * (pow(z, d) + pow(z, n - d)) / (1.0 - pow(z, n));
}

/* Offsets d and weights K(d) of one axis: the whole line when it is short. */
static int line_kernel(int n, int W, int *off, double *kw) {
  int cnt = 0;
  if (n <= 2 * W + 1) {
    for (int d = 0; d < n; ++d) { off[cnt] = d; kw[cnt] = inv_entry(n, d); ++cnt; }
  } else {
    for (int d = -W; d <= W; ++d) { off[cnt] = d; kw[cnt] = inv_entry(n, d); ++cnt; }
  }
  return cnt;
}

#define OR_WMAX 64

/* g value of component c at grid point (x, y, z) (periodic), from an FP32 or
 * FP64 field. */
static inline double field_at(const void *field, int is_f32, int64_t npts, int c, int nx,
                              int ny, int x, int y, int z) {
  const int64_t i = (int64_t)c * npts + ((int64_t)z * ny + y) * nx + x;
  return is_f32 ? (double)((const float *)field)[i] : ((const double *)field)[i];
}

/* Axis positions reached by the sums of one block: u = 0 .. U-1 stands for
 * grid index pos(u); output index k with kernel entry d reads u = uidx(k, d). */
typedef struct {
  int U, full, n, start, cnt;
} axis_win;

static axis_win make_axis(int n, int W, int a) {
  axis_win w;
  w.n = n;
  w.full = n <= 2 * W + 1;
  w.U = w.full ? n : 4 + 2 * W;
  w.start = w.full ? a - 1 : a - 1 - W;
  w.cnt = w.full ? n : 2 * W + 1;
  return w;
}

static inline int axis_pos(const axis_win *w, int u) { return wrapi(w->start + u, w->n); }
static inline int axis_u(const axis_win *w, int k, int d) {
  return w->full ? (k + d) % w->n : k + d;
}

/* The 3 x 4 x 4 x 4 coefficient block S[c][k][j][i] at grid points
 * (a0 - 1 + i, a1 - 1 + j, a2 - 1 + k) (mod n): sums along x, then y, then z,
 * each over the window of every point the next sum needs. */
static void coeff_block(const void *field, int is_f32, int nx, int ny, int nz, int W,
                        const int a[3], double blk[3][4][4][4]) {
  int off[3][2 * OR_WMAX + 1];
  double kw[3][2 * OR_WMAX + 1];
  const int n3[3] = {nx, ny, nz};
  axis_win ax[3];
  for (int d = 0; d < 3; ++d) {
    line_kernel(n3[d], W, off[d], kw[d]);
    ax[d] = make_axis(n3[d], W, a[d]);
  }
  const int64_t npts = (int64_t)nx * ny * nz;
  const int Uz = ax[2].U, Uy = ax[1].U;
  double *t1 = (double *)malloc(sizeof(double) * (size_t)Uz * Uy * 4);
  double *t2 = (double *)malloc(sizeof(double) * (size_t)Uz * 16);
  for (int c = 0; c < 3; ++c) {
    for (int uz = 0; uz < Uz; ++uz) {
      const int z = axis_pos(&ax[2], uz);
      for (int uy = 0; uy < Uy; ++uy) {
        const int y = axis_pos(&ax[1], uy);
        for (int i = 0; i < 4; ++i) {
          double sum = 0.0;
          for (int d = 0; d < ax[0].cnt; ++d) {
            const int x = axis_pos(&ax[0], axis_u(&ax[0], i, d));
            sum += kw[0][d] * field_at(field, is_f32, npts, c, nx, ny, x, y, z);
          }
          t1[((size_t)uz * Uy + uy) * 4 + i] = sum;
        }
      }
    }
    for (int uz = 0; uz < Uz; ++uz)
      for (int j = 0; j < 4; ++j)
        for (int i = 0; i < 4; ++i) {
          double sum = 0.0;
          for (int d = 0; d < ax[1].cnt; ++d)
            sum += kw[1][d] * t1[((size_t)uz * Uy + axis_u(&ax[1], j, d)) * 4 + i];
          t2[((size_t)uz * 4 + j) * 4 + i] = sum;
        }
    for (int k = 0; k < 4; ++k)
      for (int j = 0; j < 4; ++j)
        for (int i = 0; i < 4; ++i) {
          double sum = 0.0;
          for (int d = 0; d < ax[2].cnt; ++d)
            sum += kw[2][d] * t2[((size_t)axis_u(&ax[2], k, d) * 4 + j) * 4 + i];
          blk[c][k][j][i] = sum;
        }
  }
  free(t1);
  free(t2);
}

/* eq. (spline) on a coefficient block: out12 as in eval_particle. */
static void eval_block(const double blk[3][4][4][4], const double t[3], const double inv_h[3],
                       int want_grad, double *out12) {
  double w[3][4], dw[3][4];
  for (int d = 0; d < 3; ++d) {
    basis(t[d], w[d]);
    basis_dt(t[d], dw[d]);
    for (int i = 0; i < 4; ++i) dw[d][i] *= inv_h[d];
  }
  for (int q = 0; q < 12; ++q) out12[q] = 0.0;
  for (int c = 0; c < 3; ++c) {
    double v = 0, gx = 0, gy = 0, gz = 0;
    for (int k = 0; k < 4; ++k)
      for (int j = 0; j < 4; ++j)
        for (int i = 0; i < 4; ++i) {
          const double s = blk[c][k][j][i];
          v += w[0][i] * w[1][j] * w[2][k] * s;
          gx += dw[0][i] * w[1][j] * w[2][k] * s;
          gy += w[0][i] * dw[1][j] * w[2][k] * s;
          gz += w[0][i] * w[1][j] * dw[2][k] * s;
        }
    out12[c] = v;
    if (want_grad) {
      out12[3 + 3 * c + 0] = gx;
      out12[3 + 3 * c + 1] = gy;
      out12[3 + 3 * c + 2] = gz;
    }
  }
}

static void eval_window(const or_grid *gr, const void *field, int is_f32, int W,
                        const double xyz[3], int want_grad, double *out12) {
  int n[3] = {gr->nx, gr->ny, gr->nz};
  double L[3] = {gr->lx, gr->ly, gr->lz};
  int a[3];
  double t[3], inv_h[3];
  for (int d = 0; d < 3; ++d) {
    cell_1d(xyz[d], (double)n[d] / L[d], n[d], &a[d], &t[d]);
    inv_h[d] = (double)n[d] / L[d];
  }
  double blk[3][4][4][4];
  coeff_block(field, is_f32, gr->nx, gr->ny, gr->nz, W, a, blk);
  eval_block(blk, t, inv_h, want_grad, out12);
}

/* Coefficients S[c] at npt grid points pts[3][npt] (grid indices x, y, z),
 * out[3][npt]. */
int oracle_coeffs_at(int nx, int ny, int nz, const void *field, int is_f32, int W,
                     int64_t npt, const int32_t *pts, double *out) {
  if (nx < 4 || ny < 4 || nz < 4 || W < 1 || W > OR_WMAX) return OR_ERR_SIZE;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t p = 0; p < npt; ++p) {
    /* the block at a = point + 1 starts at the point itself */
    const int a[3] = {pts[p] + 1, pts[npt + p] + 1, pts[2 * npt + p] + 1};
    double blk[3][4][4][4];
    coeff_block(field, is_f32, nx, ny, nz, W, a, blk);
    for (int c = 0; c < 3; ++c) out[c * npt + p] = blk[c][0][0][0];
  }
  return OR_OK;
}

/* oracle_interp from the field itself (windowed closed-form coefficients). */
int oracle_interp_window(int nx, int ny, int nz, double lx, double ly, double lz,
                         const void *field, int is_f32, int W, int64_t np, const double *pos,
                         int n_out, double *out) {
  if (n_out != 3 && n_out != 12) return OR_ERR_SIZE;
  if (nx < 4 || ny < 4 || nz < 4 || W < 1 || W > OR_WMAX) return OR_ERR_SIZE;
  if (!check_finite(np, pos)) return OR_ERR_NONFINITE;
  or_grid gr = {nx, ny, nz, lx, ly, lz};
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t p = 0; p < np; ++p) {
    const double xyz[3] = {pos[p], pos[np + p], pos[2 * np + p]};
    double o[12];
    eval_window(&gr, field, is_f32, W, xyz, n_out == 12, o);
    for (int q = 0; q < n_out; ++q) out[q * np + p] = o[q];
  }
  return OR_OK;
}

/* nsteps Heun steps (as oracle_rk2_step) from the field itself; pos is
 * advanced in place. */
int oracle_rk2_window(int nx, int ny, int nz, double lx, double ly, double lz,
                      const void *field, int is_f32, int W, int64_t np, double dt,
                      int nsteps, double *pos) {
  if (nx < 4 || ny < 4 || nz < 4 || W < 1 || W > OR_WMAX) return OR_ERR_SIZE;
  if (!check_finite(np, pos)) return OR_ERR_NONFINITE;
  or_grid gr = {nx, ny, nz, lx, ly, lz};
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t p = 0; p < np; ++p) {
    double x0[3] = {pos[p], pos[np + p], pos[2 * np + p]};
    for (int s = 0; s < nsteps; ++s) {
      double u0[12], u1[12], xs[3];
      eval_window(&gr, field, is_f32, W, x0, 0, u0);
      for (int d = 0; d < 3; ++d) xs[d] = x0[d] + dt * u0[d];
      eval_window(&gr, field, is_f32, W, xs, 0, u1);
      for (int d = 0; d < 3; ++d) x0[d] = x0[d] + 0.5 * dt * (u0[d] + u1[d]);
    }
    for (int d = 0; d < 3; ++d) pos[d * np + p] = x0[d];
  }
  return OR_OK;
}
