/*
 * vp_oracle.c -- plain, slow FP64 CPU oracle of the six-dimensional
 * Vlasov-Poisson integrator of Yoshikawa, Yoshida & Umemura (arXiv:1206.6152):
 * directionally split positive-flux-conservative (PFC) advection, the velocity
 * moment, the FFT-convolution Poisson solve and the two-point acceleration.
 *
 * TEST INFRASTRUCTURE. Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark load this file. It shares no code, header, table or
 * constant generator with the GPU library, and the GPU library never calls it.
 *
 * Every routine follows a definition written out in the paper, in its notation
 * where possible, with no blocking, fusion or reordering:
 *   - the 1D advection step is the conservation statement of Sec. 2.1,
 *     Eq. (13): the new cell average is the integral of the reconstructed
 *     profile over the cell traced back along the characteristic. It is
 *     evaluated here as that integral (antiderivatives of the piecewise
 *     quadratic profile), not in the flux form;
 *   - the profile is the third-order reconstruction with slope correctors of
 *     the PFC scheme the paper adopts (Filbet, Sonnendrucker & Bertrand 2001);
 *   - the split step is Eq. (17), the density Eq. (18), the periodic Poisson
 *     solve Eqs. (19)-(20) by a direct (not fast) discrete Fourier transform,
 *     the isolated solve the convolution with the Green's function of Eq. (21)
 *     (direct sum, or on the doubled grid as the paper does), the acceleration
 *     Eq. (22), the time step Eqs. (23)-(25), and the diagnostics Eqs. (29),
 *     (30) and (41).
 *
 * Readings of points the paper leaves open (each also listed with the design
 * notes of the repository):
 *   R1 limiter: the slope correctors eps+/- of Filbet et al. (2001); f_inf is
 *      the maximum of the line before the sweep (Sec. 4 says the scheme needs
 *      the maximum over the whole one-dimensional region).
 *   R2 ghost cells: zero with a zero profile for outflow; wrapped for periodic.
 *   R3 periodic Poisson: the k = 0 mode of phi is zero (the expression of
 *      Eq. (20) is singular there); unequal spacings generalise Eq. (20) to
 *      -pi G / sum_l sin^2(k_l D_l / 2) / D_l^2.
 *   R4 isolated Green's function: K(r) = -G D_x D_y D_z / |r| for r != 0 and
 *      K(0) = -G times the integral of 1/|r| over one cell centred on the
 *      origin (the potential at the centre of a uniform cell of unit density).
 *      Offsets run over 0..N per axis and are mirrored on the 2N grid, so the
 *      convolution is exact for target cells -1..N, which gives the ghost
 *      potential the two-point gradient needs at the boundary.
 *   R5 force reuse: one Poisson solve per step, after the position sweeps;
 *      the first half kick of a step uses the acceleration of the previous
 *      step (or of the initial state).
 *   R6 V^max of Eq. (24) is max(|V^-|, |V^+|) per axis; an axis with zero
 *      acceleration everywhere imposes no limit in Eq. (25).
 *
 * Layout: f[ix][iy][iz][jx][jy][jz] in C order (jz fastest); the acceleration
 * is a[3][Nx*Ny*Nz]; the potential is returned with one ghost layer,
 * phi_ext[Nx+2][Ny+2][Nz+2] (index 0 is cell -1).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int32_t n[3];      /* spatial cells Nx, Ny, Nz */
  int32_t nv[3];     /* velocity cells Nvx, Nvy, Nvz */
  double L[3];       /* box lengths; space is [-L/2, L/2) */
  double vmin[3];    /* V^- per axis */
  double vmax[3];    /* V^+ per axis */
  double G;          /* gravitational constant */
  int32_t bc;        /* 0: periodic space and Poisson; 1: outflow space, isolated Poisson */
  int32_t pad;
} oracle_cfg;

static const double PI = 3.14159265358979323846;

/* ------------------------------------------------------------------ */
/* grid helpers (Sec. 2, Eqs. (3)-(4))                                */
/* ------------------------------------------------------------------ */

static double dx_of(const oracle_cfg *c, int l) { return c->L[l] / c->n[l]; }
static double dv_of(const oracle_cfg *c, int l) { return (c->vmax[l] - c->vmin[l]) / c->nv[l]; }
static double vcell(const oracle_cfg *c, int l, int j) { return c->vmin[l] + (j + 0.5) * dv_of(c, l); }

static void dims6(const oracle_cfg *c, long d[6])
{
  for (int l = 0; l < 3; l++) { d[l] = c->n[l]; d[l + 3] = c->nv[l]; }
}

static long nspace(const oracle_cfg *c) { return (long)c->n[0] * c->n[1] * c->n[2]; }
static long nvel(const oracle_cfg *c) { return (long)c->nv[0] * c->nv[1] * c->nv[2]; }

/* ------------------------------------------------------------------ */
/* one-dimensional PFC advection (Sec. 2.1)                           */
/* ------------------------------------------------------------------ */

/* value of cell k of a line of n cells, with the boundary condition of R2 */
static double line_value(const double *f, int n, long k, int periodic)
{
  if (k >= 0 && k < n) return f[k];
  if (periodic) {
    long m = k % n;
    if (m < 0) m += n;
    return f[m];
  }
  return 0.0;
}

/* Profile of cell k: mean c and the corrected one-sided differences
 *   lp = eps+ (f_{k+1} - f_k),  lm = eps- (f_k - f_{k-1}),
 * with the slope correctors of Filbet et al. (2001):
 *   eps+ = min(1, 2 f_k / (f_{k+1}-f_k))            if f_{k+1} > f_k
 *        = min(1, 2 (f_inf - f_k) / (f_k-f_{k+1}))  if f_{k+1} < f_k
 *   eps- = min(1, 2 (f_inf - f_k) / (f_k-f_{k-1}))  if f_k > f_{k-1}
 *        = min(1, 2 f_k / (f_{k-1}-f_k))            if f_k < f_{k-1}
 * limited == 0 leaves eps = 1 (the plain third-order profile; used only to
 * check the order of accuracy). Outflow ghosts have a zero profile (R2). */
static void cell_profile(const double *f, int n, long k, int periodic, double finf, int limited,
                         double *c, double *lp, double *lm)
{
  if (!periodic && (k < 0 || k >= n)) {
    *c = 0.0; *lp = 0.0; *lm = 0.0;
    return;
  }
  double fk = line_value(f, n, k, periodic);
  double dp = line_value(f, n, k + 1, periodic) - fk;
  double dm = fk - line_value(f, n, k - 1, periodic);
  double ep = 1.0, em = 1.0;
  if (limited) {
    if (dp > 0.0) ep = fmin(1.0, 2.0 * fk / dp);
    else if (dp < 0.0) ep = fmin(1.0, 2.0 * (finf - fk) / (-dp));
    if (dm > 0.0) em = fmin(1.0, 2.0 * (finf - fk) / dm);
    else if (dm < 0.0) em = fmin(1.0, 2.0 * fk / (-dm));
  }
  *c = fk;
  *lp = ep * dp;
  *lm = em * dm;
}

/* In the local coordinate s = (x - x_k)/Dx in [-1/2, 1/2] the profile is
 *   f_h(s) = c + lp (3s^2 + 3s - 1/4)/6 - lm (3s^2 - 3s - 1/4)/6,
 * the reconstruction of Filbet et al. written about the cell centre. Its
 * integral over [s0, s1] follows from the antiderivatives P and Q. */
static double anti_p(double s) { return s * s * s + 1.5 * s * s - 0.25 * s; }
static double anti_q(double s) { return s * s * s - 1.5 * s * s - 0.25 * s; }

static double profile_integral(double c, double lp, double lm, double s0, double s1)
{
  return c * (s1 - s0) + lp / 6.0 * (anti_p(s1) - anti_p(s0)) - lm / 6.0 * (anti_q(s1) - anti_q(s0));
}

/* New cell averages of one line after advection by nu = u dt / Dx cells
 * (Sec. 2.1, Eq. (13)): f'_i is the integral of f_h over
 * [x_{i-1/2} - nu Dx, x_{i+1/2} - nu Dx] divided by Dx, summed over every
 * cell the interval crosses (any |nu|; the scheme has no CFL limit, Sec. 2.4).
 * f_inf is the largest value of the line before the update (R1). */
void oracle_line(const double *f, int n, double nu, int periodic, int limited, double *out)
{
  double finf = 0.0;
  for (int i = 0; i < n; i++)
    if (f[i] > finf) finf = f[i];
  for (int i = 0; i < n; i++) {
    double a = (double)i - 0.5 - nu;
    double b = (double)i + 0.5 - nu;
    long k0 = (long)floor(a + 0.5);
    long k1 = (long)floor(b + 0.5);
    double acc = 0.0;
    for (long k = k0; k <= k1; k++) {
      double lo = fmax(a, (double)k - 0.5);
      double hi = fmin(b, (double)k + 0.5);
      if (!(hi > lo)) continue;
      double c, lp, lm;
      cell_profile(f, n, k, periodic, finf, limited, &c, &lp, &lm);
      acc += profile_integral(c, lp, lm, lo - (double)k, hi - (double)k);
    }
    out[i] = acc;
  }
}

/* Courant number of the line whose first element has flat index base
 * (Eqs. (5)-(10)): position axis l < 3 moves with v_l of the cell's velocity
 * index; velocity axis l >= 3 moves with a_{l-3} of the spatial cell. */
static double line_nu(const oracle_cfg *c, int axis, long base, double tau, const double *accel)
{
  long d[6];
  dims6(c, d);
  long idx[6], r = base;
  for (int q = 5; q >= 0; q--) { idx[q] = r % d[q]; r /= d[q]; }
  if (axis < 3) {
    return vcell(c, axis, (int)idx[axis + 3]) * tau / dx_of(c, axis);
  }
  long sp = (idx[0] * d[1] + idx[1]) * d[2] + idx[2];
  int l = axis - 3;
  return accel[(long)l * nspace(c) + sp] * tau / dv_of(c, l);
}

/* One directional sweep T_axis(tau) over every line of f (axis 0..2 = x, y, z;
 * 3..5 = vx, vy, vz). Velocity axes are outflow (Sec. 2.1); position axes are
 * periodic when bc == 0 and outflow otherwise. accel may be NULL for position
 * axes. */
void oracle_sweep(const oracle_cfg *c, double *f, int axis, double tau, const double *accel)
{
  long d[6];
  dims6(c, d);
  long stride = 1;
  for (int q = 5; q > axis; q--) stride *= d[q];
  long n = d[axis];
  long outer = 1;
  for (int q = 0; q < axis; q++) outer *= d[q];
  int periodic = (axis < 3 && c->bc == 0);
  long nlines = outer * stride;
#pragma omp parallel
  {
    double *in = (double *)malloc(sizeof(double) * n);
    double *out = (double *)malloc(sizeof(double) * n);
#pragma omp for schedule(static)
    for (long line = 0; line < nlines; line++) {
      long o = line / stride, cidx = line % stride;
      long base = o * n * stride + cidx;
      for (long i = 0; i < n; i++) in[i] = f[base + i * stride];
      double nu = line_nu(c, axis, base, tau, accel);
      oracle_line(in, (int)n, nu, periodic, 1, out);
      for (long i = 0; i < n; i++) f[base + i * stride] = out[i];
    }
    free(in);
    free(out);
  }
}

/* ------------------------------------------------------------------ */
/* gravity (Sec. 2.2)                                                 */
/* ------------------------------------------------------------------ */

/* rho(x) = integral of f over velocity (Eq. (18)), midpoint sum in fixed order */
void oracle_density(const oracle_cfg *c, const double *f, double *rho)
{
  long np = nspace(c), nv = nvel(c);
  double dv3 = dv_of(c, 0) * dv_of(c, 1) * dv_of(c, 2);
  for (long s = 0; s < np; s++) {
    double acc = 0.0;
    for (long j = 0; j < nv; j++) acc += f[s * nv + j];
    rho[s] = acc * dv3;
  }
}

/* Direct discrete Fourier transform along one axis of a complex field of
 * shape m[0] x m[1] x m[2] (C order), in place: X_k = sum_j x_j
 * exp(sign 2 pi i j k / M), no scaling. Twiddle angles use (j k mod M). */
static void dft_axis(double *re, double *im, const long m[3], int axis, int sign)
{
  long M = m[axis];
  long stride = 1;
  for (int q = 2; q > axis; q--) stride *= m[q];
  long outer = 1;
  for (int q = 0; q < axis; q++) outer *= m[q];
  long nlines = outer * stride;
#pragma omp parallel
  {
    double *xr = (double *)malloc(sizeof(double) * M);
    double *xi = (double *)malloc(sizeof(double) * M);
#pragma omp for schedule(static)
    for (long line = 0; line < nlines; line++) {
      long o = line / stride, cidx = line % stride;
      long base = o * M * stride + cidx;
      for (long j = 0; j < M; j++) { xr[j] = re[base + j * stride]; xi[j] = im[base + j * stride]; }
      for (long k = 0; k < M; k++) {
        double sr = 0.0, si = 0.0;
        for (long j = 0; j < M; j++) {
          double ang = sign * 2.0 * PI * (double)((j * k) % M) / (double)M;
          double cr = cos(ang), ci = sin(ang);
          sr += xr[j] * cr - xi[j] * ci;
          si += xr[j] * ci + xi[j] * cr;
        }
        re[base + k * stride] = sr;
        im[base + k * stride] = si;
      }
    }
    free(xr);
    free(xi);
  }
}

static long ext_index(const oracle_cfg *c, long i0, long i1, long i2)
{
  /* position (i0, i1, i2), each in -1..N, in the ghost-padded array */
  return ((i0 + 1) * (c->n[1] + 2) + (i1 + 1)) * (c->n[2] + 2) + (i2 + 1);
}

/* Periodic potential: phi_hat = G_hat rho_hat (Eqs. (19)-(20), reading R3),
 * by the direct DFT, returned with wrapped ghost cells. */
static void potential_periodic(const oracle_cfg *c, const double *rho, double *phi_ext)
{
  long m[3] = {c->n[0], c->n[1], c->n[2]};
  long np = nspace(c);
  double *re = (double *)calloc(np, sizeof(double));
  double *im = (double *)calloc(np, sizeof(double));
  for (long s = 0; s < np; s++) re[s] = rho[s];
  for (int ax = 0; ax < 3; ax++) dft_axis(re, im, m, ax, -1);
  double d[3] = {dx_of(c, 0), dx_of(c, 1), dx_of(c, 2)};
  for (long k0 = 0; k0 < m[0]; k0++)
    for (long k1 = 0; k1 < m[1]; k1++)
      for (long k2 = 0; k2 < m[2]; k2++) {
        long s = (k0 * m[1] + k1) * m[2] + k2;
        double s0 = sin(PI * k0 / m[0]), s1 = sin(PI * k1 / m[1]), s2 = sin(PI * k2 / m[2]);
        double den = s0 * s0 / (d[0] * d[0]) + s1 * s1 / (d[1] * d[1]) + s2 * s2 / (d[2] * d[2]);
        double g = (k0 == 0 && k1 == 0 && k2 == 0) ? 0.0 : -PI * c->G / den;
        re[s] *= g;
        im[s] *= g;
      }
  for (int ax = 0; ax < 3; ax++) dft_axis(re, im, m, ax, +1);
  for (long i0 = -1; i0 <= m[0]; i0++)
    for (long i1 = -1; i1 <= m[1]; i1++)
      for (long i2 = -1; i2 <= m[2]; i2++) {
        long w0 = (i0 + m[0]) % m[0], w1 = (i1 + m[1]) % m[1], w2 = (i2 + m[2]) % m[2];
        phi_ext[ext_index(c, i0, i1, i2)] = re[(w0 * m[1] + w1) * m[2] + w2] / (double)np;
      }
  free(re);
  free(im);
}

/* Integral of 1/|r| over the box [0,a]x[0,b]x[0,c] (one corner at the origin),
 * the closed form for the potential of a uniform rectangular box at a corner. */
static double corner_integral(double a, double b, double c)
{
  double d = sqrt(a * a + b * b + c * c);
  return a * b * log((c + d) / sqrt(a * a + b * b)) + b * c * log((a + d) / sqrt(b * b + c * c)) +
         c * a * log((b + d) / sqrt(c * c + a * a)) - 0.5 * a * a * atan(b * c / (a * d)) -
         0.5 * b * b * atan(c * a / (b * d)) - 0.5 * c * c * atan(a * b / (c * d));
}

/* Integral of 1/|r| over one cell centred on the origin (reading R4). */
double oracle_cell_self_integral(double dx, double dy, double dz)
{
  return 8.0 * corner_integral(0.5 * dx, 0.5 * dy, 0.5 * dz);
}

/* Green's function of reading R4 at integer offset (m0, m1, m2). */
static double green_isolated(const oracle_cfg *c, long m0, long m1, long m2)
{
  double d0 = dx_of(c, 0), d1 = dx_of(c, 1), d2 = dx_of(c, 2);
  if (m0 == 0 && m1 == 0 && m2 == 0) return -c->G * oracle_cell_self_integral(d0, d1, d2);
  double r = sqrt((m0 * d0) * (m0 * d0) + (m1 * d1) * (m1 * d1) + (m2 * d2) * (m2 * d2));
  return -c->G * d0 * d1 * d2 / r;
}

/* Isolated potential as the plain convolution sum phi(t) = sum_i K(t-i) rho_i
 * over target cells t in -1..N (Eq. (21), reading R4). O(N^6). */
void oracle_potential_isolated_direct(const oracle_cfg *c, const double *rho, double *phi_ext)
{
  long n0 = c->n[0], n1 = c->n[1], n2 = c->n[2];
#pragma omp parallel for collapse(2) schedule(static)
  for (long t0 = -1; t0 <= n0; t0++)
    for (long t1 = -1; t1 <= n1; t1++)
      for (long t2 = -1; t2 <= n2; t2++) {
        double acc = 0.0;
        for (long i0 = 0; i0 < n0; i0++)
          for (long i1 = 0; i1 < n1; i1++)
            for (long i2 = 0; i2 < n2; i2++)
              acc += green_isolated(c, t0 - i0, t1 - i1, t2 - i2) * rho[(i0 * n1 + i1) * n2 + i2];
        phi_ext[ext_index(c, t0, t1, t2)] = acc;
      }
}

/* Isolated potential by the doubling-up method the paper uses (Sec. 2.2):
 * zero-pad rho to 2N per axis, mirror the Green's function of offsets 0..N
 * into a 2N-periodic kernel, multiply the (direct) DFTs, transform back. */
void oracle_potential_isolated_doubled(const oracle_cfg *c, const double *rho, double *phi_ext)
{
  long m[3] = {2L * c->n[0], 2L * c->n[1], 2L * c->n[2]};
  long tot = m[0] * m[1] * m[2];
  double *rr = (double *)calloc(tot, sizeof(double));
  double *ri = (double *)calloc(tot, sizeof(double));
  double *kr = (double *)calloc(tot, sizeof(double));
  double *ki = (double *)calloc(tot, sizeof(double));
  for (long i0 = 0; i0 < c->n[0]; i0++)
    for (long i1 = 0; i1 < c->n[1]; i1++)
      for (long i2 = 0; i2 < c->n[2]; i2++)
        rr[(i0 * m[1] + i1) * m[2] + i2] = rho[(i0 * c->n[1] + i1) * c->n[2] + i2];
  for (long o0 = 0; o0 < m[0]; o0++)
    for (long o1 = 0; o1 < m[1]; o1++)
      for (long o2 = 0; o2 < m[2]; o2++) {
        long a0 = o0 < m[0] - o0 ? o0 : m[0] - o0;
        long a1 = o1 < m[1] - o1 ? o1 : m[1] - o1;
        long a2 = o2 < m[2] - o2 ? o2 : m[2] - o2;
        kr[(o0 * m[1] + o1) * m[2] + o2] = green_isolated(c, a0, a1, a2);
      }
  for (int ax = 0; ax < 3; ax++) {
    dft_axis(rr, ri, m, ax, -1);
    dft_axis(kr, ki, m, ax, -1);
  }
  for (long s = 0; s < tot; s++) {
    double a = rr[s] * kr[s] - ri[s] * ki[s];
    double b = rr[s] * ki[s] + ri[s] * kr[s];
    rr[s] = a;
    ri[s] = b;
  }
  for (int ax = 0; ax < 3; ax++) dft_axis(rr, ri, m, ax, +1);
  for (long t0 = -1; t0 <= c->n[0]; t0++)
    for (long t1 = -1; t1 <= c->n[1]; t1++)
      for (long t2 = -1; t2 <= c->n[2]; t2++) {
        long w0 = (t0 + m[0]) % m[0], w1 = (t1 + m[1]) % m[1], w2 = (t2 + m[2]) % m[2];
        phi_ext[ext_index(c, t0, t1, t2)] = rr[(w0 * m[1] + w1) * m[2] + w2] / (double)tot;
      }
  free(rr);
  free(ri);
  free(kr);
  free(ki);
}

/* Potential with one ghost layer: periodic or isolated per the boundary type.
 * The isolated case uses the plain sum on small grids and the doubled-grid
 * transform otherwise; the two agree to rounding (checked by the tests). */
void oracle_potential(const oracle_cfg *c, const double *rho, double *phi_ext)
{
  if (c->bc == 0) {
    potential_periodic(c, rho, phi_ext);
  } else {
    double work = (double)(c->n[0] + 2) * (c->n[1] + 2) * (c->n[2] + 2) * (double)nspace(c);
    if (work <= 3.0e7) oracle_potential_isolated_direct(c, rho, phi_ext);
    else oracle_potential_isolated_doubled(c, rho, phi_ext);
  }
}

/* a = -grad phi by the two-point difference of Eq. (22). */
void oracle_accel_from_phi(const oracle_cfg *c, const double *phi_ext, double *accel)
{
  long n0 = c->n[0], n1 = c->n[1], n2 = c->n[2], np = nspace(c);
  double d[3] = {dx_of(c, 0), dx_of(c, 1), dx_of(c, 2)};
  for (long i0 = 0; i0 < n0; i0++)
    for (long i1 = 0; i1 < n1; i1++)
      for (long i2 = 0; i2 < n2; i2++) {
        long s = (i0 * n1 + i1) * n2 + i2;
        accel[0 * np + s] = -(phi_ext[ext_index(c, i0 + 1, i1, i2)] - phi_ext[ext_index(c, i0 - 1, i1, i2)]) / (2.0 * d[0]);
        accel[1 * np + s] = -(phi_ext[ext_index(c, i0, i1 + 1, i2)] - phi_ext[ext_index(c, i0, i1 - 1, i2)]) / (2.0 * d[1]);
        accel[2 * np + s] = -(phi_ext[ext_index(c, i0, i1, i2 + 1)] - phi_ext[ext_index(c, i0, i1, i2 - 1)]) / (2.0 * d[2]);
      }
}

static long ext_size(const oracle_cfg *c) { return (long)(c->n[0] + 2) * (c->n[1] + 2) * (c->n[2] + 2); }

/* density -> potential -> acceleration from the current f */
void oracle_accel(const oracle_cfg *c, const double *f, double *accel)
{
  double *rho = (double *)malloc(sizeof(double) * nspace(c));
  double *phi = (double *)malloc(sizeof(double) * ext_size(c));
  oracle_density(c, f, rho);
  oracle_potential(c, rho, phi);
  oracle_accel_from_phi(c, phi, accel);
  free(rho);
  free(phi);
}

/* ------------------------------------------------------------------ */
/* time integration (Sec. 2.1, Eq. (17); Sec. 2.4)                    */
/* ------------------------------------------------------------------ */

/* One step of Eq. (17): T_vx, T_vy, T_vz at dt/2 with the acceleration held
 * in accel; T_z, T_y, T_x at dt; then the Poisson solve (which overwrites
 * accel); then T_vx, T_vy, T_vz at dt/2 (reading R5). */
void oracle_step(const oracle_cfg *c, double *f, double dt, double *accel)
{
  oracle_sweep(c, f, 3, 0.5 * dt, accel);
  oracle_sweep(c, f, 4, 0.5 * dt, accel);
  oracle_sweep(c, f, 5, 0.5 * dt, accel);
  oracle_sweep(c, f, 2, dt, NULL);
  oracle_sweep(c, f, 1, dt, NULL);
  oracle_sweep(c, f, 0, dt, NULL);
  oracle_accel(c, f, accel);
  oracle_sweep(c, f, 3, 0.5 * dt, accel);
  oracle_sweep(c, f, 4, 0.5 * dt, accel);
  oracle_sweep(c, f, 5, 0.5 * dt, accel);
}

/* dt = C min(dt_p, dt_v), Eqs. (23)-(25) with reading R6. */
double oracle_dt(const oracle_cfg *c, const double *accel, double cfl)
{
  double dtp = INFINITY, dtv = INFINITY;
  for (int l = 0; l < 3; l++) {
    double vm = fmax(fabs(c->vmin[l]), fabs(c->vmax[l]));
    if (vm > 0.0) dtp = fmin(dtp, dx_of(c, l) / vm);
  }
  long np = nspace(c);
  for (int l = 0; l < 3; l++)
    for (long s = 0; s < np; s++) {
      double a = fabs(accel[(long)l * np + s]);
      if (a > 0.0) dtv = fmin(dtv, dv_of(c, l) / a);
    }
  return cfl * fmin(dtp, dtv);
}

/* K, U, M, E (Eqs. (29), (30), (41)) with cell-centre velocities. */
void oracle_energy(const oracle_cfg *c, const double *f, double out[4])
{
  long np = nspace(c);
  double dx3 = dx_of(c, 0) * dx_of(c, 1) * dx_of(c, 2);
  double dv3 = dv_of(c, 0) * dv_of(c, 1) * dv_of(c, 2);
  double kin = 0.0, mass = 0.0;
  for (long s = 0; s < np; s++)
    for (int jx = 0; jx < c->nv[0]; jx++)
      for (int jy = 0; jy < c->nv[1]; jy++)
        for (int jz = 0; jz < c->nv[2]; jz++) {
          double vx = vcell(c, 0, jx), vy = vcell(c, 1, jy), vz = vcell(c, 2, jz);
          double v = f[((s * c->nv[0] + jx) * c->nv[1] + jy) * c->nv[2] + jz];
          mass += v;
          kin += 0.5 * v * (vx * vx + vy * vy + vz * vz);
        }
  double *rho = (double *)malloc(sizeof(double) * np);
  double *phi = (double *)malloc(sizeof(double) * ext_size(c));
  oracle_density(c, f, rho);
  oracle_potential(c, rho, phi);
  double pot = 0.0;
  for (long i0 = 0; i0 < c->n[0]; i0++)
    for (long i1 = 0; i1 < c->n[1]; i1++)
      for (long i2 = 0; i2 < c->n[2]; i2++)
        pot += 0.5 * rho[(i0 * c->n[1] + i1) * c->n[2] + i2] * phi[ext_index(c, i0, i1, i2)];
  free(rho);
  free(phi);
  out[0] = kin * dx3 * dv3;
  out[1] = pot * dx3;
  out[2] = mass * dx3 * dv3;
  out[3] = out[0] + out[1];
}

/* number of OpenMP threads the oracle runs on (1 without OpenMP) */
int oracle_num_threads(void)
{
#ifdef _OPENMP
  extern int omp_get_max_threads(void);
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* reverse mode (gradient of the field energy; not in the paper)      */
/* ------------------------------------------------------------------ */
/*
 * The loss is L = -U of the final state (U of Eq. (41)), a function of the
 * initial f through nsteps steps of Eq. (17) with a fixed dt. The reverse mode
 * below is written against this file's own forward definitions:
 *   - the line update is the integral of the limited profile over the
 *     traced-back interval, out_i = sum over crossed cells k of
 *     c_k w0 + lp_k w1 - lm_k w2 with weights that depend only on nu; its
 *     adjoint sends lam_out through those weights to (c, lp, lm), then through
 *     the corrector branch that is active (a corrector that bounds the slope
 *     by 2 f_k or by 2 (f_inf - f_k) passes the adjoint to f_k and to f_inf),
 *     and f_inf passes its adjoint to the first cell holding the maximum;
 *   - the derivative in nu is the Leibniz rule at the two ends of the
 *     traced-back interval: d out_i / d nu = f_h(left end) - f_h(right end);
 *   - a velocity sweep's nu = a_l(x) tau / dv_l carries the adjoint to a_l;
 *   - the acceleration, potential and density are linear; their transposes
 *     are written out (the periodic operator and the isolated convolution
 *     are symmetric).
 * Branch convention at exact ties: a corrector bound is active only when the
 * one-sided difference is strictly beyond it.
 */

static double profile_value(double c, double lp, double lm, double s)
{
  return c + lp * (3.0 * s * s + 3.0 * s - 0.25) / 6.0 - lm * (3.0 * s * s - 3.0 * s - 0.25) / 6.0;
}

static long wrap_index(long k, int n) { long m = k % n; return m < 0 ? m + n : m; }

/* Adjoint of oracle_line: lam_f += J^T lam_out (J = d out / d f); returns
 * sum_i lam_out_i d out_i / d nu. */
double oracle_line_vjp(const double *f, int n, double nu, int periodic, const double *lam_out, double *lam_f)
{
  double finf = 0.0;
  int amax = -1;
  for (int i = 0; i < n; i++)
    if (f[i] > finf) { finf = f[i]; amax = i; }
  double *lc = (double *)calloc(n, sizeof(double));
  double *lp_ = (double *)calloc(n, sizeof(double));
  double *lm_ = (double *)calloc(n, sizeof(double));
  double dnu = 0.0;
  for (int i = 0; i < n; i++) {
    if (lam_out[i] == 0.0) continue;
    double a = (double)i - 0.5 - nu;
    double b = (double)i + 0.5 - nu;
    long k0 = (long)floor(a + 0.5);
    long k1 = (long)floor(b + 0.5);
    for (long k = k0; k <= k1; k++) {
      double lo = fmax(a, (double)k - 0.5);
      double hi = fmin(b, (double)k + 0.5);
      if (!(hi > lo)) continue;
      if (!periodic && (k < 0 || k >= n)) continue;   /* zero profile */
      long kk = periodic ? wrap_index(k, n) : k;
      double s0 = lo - (double)k, s1 = hi - (double)k;
      double c, lp, lm;
      cell_profile(f, n, k, periodic, finf, 1, &c, &lp, &lm);
      lc[kk] += lam_out[i] * (s1 - s0);
      lp_[kk] += lam_out[i] * (anti_p(s1) - anti_p(s0)) / 6.0;
      lm_[kk] -= lam_out[i] * (anti_q(s1) - anti_q(s0)) / 6.0;
      if (lo == a) dnu += lam_out[i] * profile_value(c, lp, lm, s0);
      if (hi == b) dnu -= lam_out[i] * profile_value(c, lp, lm, s1);
    }
  }
  double lfinf = 0.0;
  for (int k = 0; k < n; k++) {
    double fk = f[k];
    long kr = k + 1, kl = k - 1;
    int has_r = periodic || kr < n, has_l = periodic || kl >= 0;
    double fr = has_r ? f[periodic ? wrap_index(kr, n) : kr] : 0.0;
    double fl = has_l ? f[periodic ? wrap_index(kl, n) : kl] : 0.0;
    lam_f[k] += lc[k];
    /* lp = eps+ (f_{k+1} - f_k) */
    double dp = fr - fk, g = lp_[k];
    if (dp > 0.0 && 2.0 * fk < dp) {
      lam_f[k] += 2.0 * g;
    } else if (dp < 0.0 && 2.0 * (finf - fk) < -dp) {
      lfinf -= 2.0 * g;
      lam_f[k] += 2.0 * g;
    } else {
      if (has_r) lam_f[periodic ? wrap_index(kr, n) : kr] += g;
      lam_f[k] -= g;
    }
    /* lm = eps- (f_k - f_{k-1}) */
    double dm = fk - fl;
    g = lm_[k];
    if (dm > 0.0 && 2.0 * (finf - fk) < dm) {
      lfinf += 2.0 * g;
      lam_f[k] -= 2.0 * g;
    } else if (dm < 0.0 && 2.0 * fk < -dm) {
      lam_f[k] -= 2.0 * g;
    } else {
      lam_f[k] += g;
      if (has_l) lam_f[periodic ? wrap_index(kl, n) : kl] -= g;
    }
  }
  if (amax >= 0) lam_f[amax] += lfinf;
  free(lc);
  free(lp_);
  free(lm_);
  return dnu;
}

/* Adjoint of oracle_sweep at input state f_in: lam <- J^T lam; for velocity
 * axes lam_accel[axis-3][x] += (tau / dv) * (sum over the cell's lines of the
 * nu-adjoint). */
void oracle_sweep_vjp(const oracle_cfg *c, const double *f_in, int axis, double tau, const double *accel,
                      double *lam, double *lam_accel)
{
  long d[6];
  dims6(c, d);
  long stride = 1;
  for (int q = 5; q > axis; q--) stride *= d[q];
  long n = d[axis];
  long outer = 1;
  for (int q = 0; q < axis; q++) outer *= d[q];
  int periodic = (axis < 3 && c->bc == 0);
  long nlines = outer * stride;
  long np = nspace(c);
  double *dnu_line = (double *)calloc(nlines, sizeof(double));
#pragma omp parallel
  {
    double *in = (double *)malloc(sizeof(double) * n);
    double *lo = (double *)malloc(sizeof(double) * n);
    double *li = (double *)malloc(sizeof(double) * n);
#pragma omp for schedule(static)
    for (long line = 0; line < nlines; line++) {
      long o = line / stride, cidx = line % stride;
      long base = o * n * stride + cidx;
      for (long i = 0; i < n; i++) {
        in[i] = f_in[base + i * stride];
        lo[i] = lam[base + i * stride];
        li[i] = 0.0;
      }
      double nu = line_nu(c, axis, base, tau, accel);
      dnu_line[line] = oracle_line_vjp(in, (int)n, nu, periodic, lo, li);
      for (long i = 0; i < n; i++) lam[base + i * stride] = li[i];
    }
    free(in);
    free(lo);
    free(li);
  }
  if (axis >= 3 && lam_accel) {
    int l = axis - 3;
    double sc = tau / dv_of(c, l);
    /* lines of spatial cell s: outer index o = s * (lines of preceding velocity axes) + ... */
    long per = outer / np;  /* slabs per spatial cell */
    for (long line = 0; line < nlines; line++) {
      long o = line / stride;
      long s = o / per;
      lam_accel[(long)l * np + s] += sc * dnu_line[line];
    }
  }
  free(dnu_line);
}

/* Adjoint of density -> potential -> acceleration at any state:
 * lam_f[x, v] += dv3 * lam_rho[x], lam_rho = G_ext^T D^T lam_accel. */
void oracle_accel_vjp(const oracle_cfg *c, const double *lam_accel, double *lam_f)
{
  long n0 = c->n[0], n1 = c->n[1], n2 = c->n[2], np = nspace(c), nv = nvel(c);
  double d[3] = {dx_of(c, 0), dx_of(c, 1), dx_of(c, 2)};
  long ne = ext_size(c);
  double *lphi = (double *)calloc(ne, sizeof(double));
  /* D^T: a_l(i) = -(phi(i+e_l) - phi(i-e_l)) / (2 d_l) */
  for (long i0 = 0; i0 < n0; i0++)
    for (long i1 = 0; i1 < n1; i1++)
      for (long i2 = 0; i2 < n2; i2++) {
        long s = (i0 * n1 + i1) * n2 + i2;
        double g0 = lam_accel[s] / (2.0 * d[0]);
        double g1 = lam_accel[np + s] / (2.0 * d[1]);
        double g2 = lam_accel[2 * np + s] / (2.0 * d[2]);
        lphi[ext_index(c, i0 + 1, i1, i2)] -= g0;
        lphi[ext_index(c, i0 - 1, i1, i2)] += g0;
        lphi[ext_index(c, i0, i1 + 1, i2)] -= g1;
        lphi[ext_index(c, i0, i1 - 1, i2)] += g1;
        lphi[ext_index(c, i0, i1, i2 + 1)] -= g2;
        lphi[ext_index(c, i0, i1, i2 - 1)] += g2;
      }
  double *lrho = (double *)calloc(np, sizeof(double));
  if (c->bc == 0) {
    /* ghosts are periodic images: fold, then apply the symmetric operator */
    double *fold = (double *)calloc(np, sizeof(double));
    for (long t0 = -1; t0 <= n0; t0++)
      for (long t1 = -1; t1 <= n1; t1++)
        for (long t2 = -1; t2 <= n2; t2++) {
          long w0 = (t0 + n0) % n0, w1 = (t1 + n1) % n1, w2 = (t2 + n2) % n2;
          fold[(w0 * n1 + w1) * n2 + w2] += lphi[ext_index(c, t0, t1, t2)];
        }
    double *tmp = (double *)malloc(sizeof(double) * ne);
    potential_periodic(c, fold, tmp);
    for (long i0 = 0; i0 < n0; i0++)
      for (long i1 = 0; i1 < n1; i1++)
        for (long i2 = 0; i2 < n2; i2++) lrho[(i0 * n1 + i1) * n2 + i2] = tmp[ext_index(c, i0, i1, i2)];
    free(fold);
    free(tmp);
  } else {
    /* lam_rho(i) = sum over targets t in -1..N of K(t - i) lam_phi(t) */
    for (long i0 = 0; i0 < n0; i0++)
      for (long i1 = 0; i1 < n1; i1++)
        for (long i2 = 0; i2 < n2; i2++) {
          double acc = 0.0;
          for (long t0 = -1; t0 <= n0; t0++)
            for (long t1 = -1; t1 <= n1; t1++)
              for (long t2 = -1; t2 <= n2; t2++) {
                double g = lphi[ext_index(c, t0, t1, t2)];
                if (g != 0.0) acc += green_isolated(c, t0 - i0, t1 - i1, t2 - i2) * g;
              }
          lrho[(i0 * n1 + i1) * n2 + i2] = acc;
        }
  }
  double dv3 = dv_of(c, 0) * dv_of(c, 1) * dv_of(c, 2);
  for (long s = 0; s < np; s++)
    for (long j = 0; j < nv; j++) lam_f[s * nv + j] += dv3 * lrho[s];
  free(lphi);
  free(lrho);
}

/* L = -U(f_N) after nsteps steps of Eq. (17) from f0 with fixed dt; writes
 * dL/df0 into grad (layout of f) and returns L. Keeps every intermediate
 * state, so it is meant for small grids. */
double oracle_grad(const oracle_cfg *c, const double *f0, int nsteps, double dt, double *grad)
{
  long np = nspace(c), nv = nvel(c), nc = np * nv;
  const int axes[10] = {3, 4, 5, 2, 1, 0, -1, 3, 4, 5};
  /* states[n][k] = input of the k-th sweep of step n (k = 0..8) */
  double **st = (double **)malloc(sizeof(double *) * (size_t)nsteps * 9);
  double **acc = (double **)malloc(sizeof(double *) * (size_t)(nsteps + 1));
  double *f = (double *)malloc(sizeof(double) * nc);
  memcpy(f, f0, sizeof(double) * nc);
  acc[0] = (double *)malloc(sizeof(double) * 3 * np);
  oracle_accel(c, f, acc[0]);
  for (int n = 0; n < nsteps; n++) {
    int k = 0;
    for (int q = 0; q < 10; q++) {
      if (axes[q] < 0) {
        acc[n + 1] = (double *)malloc(sizeof(double) * 3 * np);
        oracle_accel(c, f, acc[n + 1]);
        continue;
      }
      st[n * 9 + k] = (double *)malloc(sizeof(double) * nc);
      memcpy(st[n * 9 + k], f, sizeof(double) * nc);
      k++;
      double tau = axes[q] >= 3 ? 0.5 * dt : dt;
      oracle_sweep(c, f, axes[q], tau, q < 6 ? acc[n] : acc[n + 1]);
    }
  }
  /* loss and seed */
  double *rho = (double *)malloc(sizeof(double) * np);
  double *phi = (double *)malloc(sizeof(double) * ext_size(c));
  oracle_density(c, f, rho);
  oracle_potential(c, rho, phi);
  double dx3 = dx_of(c, 0) * dx_of(c, 1) * dx_of(c, 2);
  double dv3 = dv_of(c, 0) * dv_of(c, 1) * dv_of(c, 2);
  double U = 0.0;
  for (long i0 = 0; i0 < c->n[0]; i0++)
    for (long i1 = 0; i1 < c->n[1]; i1++)
      for (long i2 = 0; i2 < c->n[2]; i2++) {
        long s = (i0 * c->n[1] + i1) * c->n[2] + i2;
        U += 0.5 * rho[s] * phi[ext_index(c, i0, i1, i2)] * dx3;
        for (long j = 0; j < nv; j++) grad[s * nv + j] = -dx3 * dv3 * phi[ext_index(c, i0, i1, i2)];
      }
  double *lam_pending = (double *)calloc(3 * np, sizeof(double));
  double *lam_a = (double *)calloc(3 * np, sizeof(double));
  for (int n = nsteps - 1; n >= 0; n--) {
    /* second half kick of step n (acceleration a_{n+1}) */
    memcpy(lam_a, lam_pending, sizeof(double) * 3 * np);
    for (int k = 8; k >= 6; k--) oracle_sweep_vjp(c, st[n * 9 + k], axes[k + 1], 0.5 * dt, acc[n + 1], grad, lam_a);
    /* a_{n+1} = A(state after the drift) */
    oracle_accel_vjp(c, lam_a, grad);
    /* drift */
    for (int k = 5; k >= 3; k--) oracle_sweep_vjp(c, st[n * 9 + k], axes[k], dt, NULL, grad, NULL);
    /* first half kick (acceleration a_n) */
    memset(lam_pending, 0, sizeof(double) * 3 * np);
    for (int k = 2; k >= 0; k--) oracle_sweep_vjp(c, st[n * 9 + k], axes[k], 0.5 * dt, acc[n], grad, lam_pending);
  }
  /* a_0 = A(f0) */
  oracle_accel_vjp(c, lam_pending, grad);
  for (long i = 0; i < (long)nsteps * 9; i++) free(st[i]);
  for (int n = 0; n <= nsteps; n++) free(acc[n]);
  free(st);
  free(acc);
  free(f);
  free(rho);
  free(phi);
  free(lam_pending);
  free(lam_a);
  return -U;
}

/* L = -U of f (the loss itself, for finite differences) */
double oracle_field_energy_loss(const oracle_cfg *c, const double *f)
{
  double e[4];
  oracle_energy(c, f, e);
  return -e[1];
}
