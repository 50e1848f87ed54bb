/*
 * Runs every routine of the FP64 oracle once or more on small periodic and
 * outflow/isolated grids, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitized_builds.py). The oracle is
 * included as source so that its static helpers are instrumented too. The
 * values are summed into a checksum that is printed, so that no call is
 * optimised away; correctness is pinned elsewhere. Built with -DPLANT_OOB it
 * reads one element past an array, which the sanitizer must report.
 */
#include "vp_oracle.c"

#include <stdio.h>

static uint64_t lcg = 88172645463325252ull;
static double urand(void)
{
  lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
  return (double)(lcg >> 11) * (1.0 / 9007199254740992.0);
}

static double sum(const double *x, long n)
{
  double s = 0.0;
  for (long i = 0; i < n; i++) s += x[i];
  return s;
}

static double exercise(const oracle_cfg *c, double *checksum)
{
  const long np = nspace(c), nv = nvel(c), nc = np * nv, ne = ext_size(c);
  double *f = malloc(sizeof(double) * nc), *g = malloc(sizeof(double) * nc);
  double *lam = malloc(sizeof(double) * nc), *grad = malloc(sizeof(double) * nc);
  double *rho = malloc(sizeof(double) * np), *phi = malloc(sizeof(double) * ne);
  double *acc = malloc(sizeof(double) * 3 * np), *lacc = calloc(3 * np, sizeof(double));
  double e[4];
  for (long i = 0; i < nc; i++) f[i] = 0.05 + urand();
  oracle_density(c, f, rho);
  oracle_potential(c, rho, phi);
  *checksum += sum(phi, ne);
  if (c->bc == 1) {
    oracle_potential_isolated_direct(c, rho, phi);
    *checksum += sum(phi, ne);
    oracle_potential_isolated_doubled(c, rho, phi);
    *checksum += sum(phi, ne);
  }
  oracle_accel_from_phi(c, phi, acc);
  oracle_accel(c, f, acc);
  *checksum += sum(acc, 3 * np);
  /* every axis, with Courant numbers past one cell */
  for (int axis = 0; axis < 6; axis++) {
    memcpy(g, f, sizeof(double) * nc);
    oracle_sweep(c, g, axis, axis < 3 ? 0.6 : 0.9, acc);
    *checksum += sum(g, nc);
    for (long i = 0; i < nc; i++) lam[i] = urand() - 0.5;
    oracle_sweep_vjp(c, f, axis, axis < 3 ? 0.6 : 0.9, acc, lam, lacc);
    *checksum += sum(lam, nc) + sum(lacc, 3 * np);
  }
  for (long i = 0; i < 3 * np; i++) lacc[i] = urand() - 0.5;
  memset(lam, 0, sizeof(double) * nc);
  oracle_accel_vjp(c, lacc, lam);
  *checksum += sum(lam, nc);
  memcpy(g, f, sizeof(double) * nc);
  oracle_step(c, g, 0.05, acc);
  oracle_step(c, g, 0.05, acc);
  *checksum += sum(g, nc) + oracle_dt(c, acc, 0.5);
  oracle_energy(c, g, e);
  *checksum += e[0] + e[1] + e[2] + e[3];
  const double loss = oracle_grad(c, f, 2, 0.05, grad);
  *checksum += loss + sum(grad, nc) + oracle_field_energy_loss(c, f);
#ifdef PLANT_OOB
  *checksum += f[nc]; /* one past the end: the sanitizer must report it */
#endif
  free(f);
  free(g);
  free(lam);
  free(grad);
  free(rho);
  free(phi);
  free(acc);
  free(lacc);
  return *checksum;
}

int main(void)
{
  double checksum = 0.0;
  /* single lines: both boundaries, limited and not, shifts of both signs */
  const double nus[] = {-2.7, -1.0, -0.3, 0.0, 0.4, 1.0, 1.9};
  const int lens[] = {1, 2, 3, 7};
  for (int li = 0; li < 4; li++) {
    const int n = lens[li];
    double f[7], out[7], lo[7], lf[7];
    for (int i = 0; i < n; i++) {
      f[i] = (i % 3 == 0) ? 0.0 : urand();
      lo[i] = urand() - 0.5;
    }
    for (int k = 0; k < 7; k++)
      for (int periodic = 0; periodic < 2; periodic++) {
        for (int limited = 0; limited < 2; limited++) {
          oracle_line(f, n, nus[k], periodic, limited, out);
          checksum += sum(out, n);
        }
        memset(lf, 0, sizeof lf);
        checksum += oracle_line_vjp(f, n, nus[k], periodic, lo, lf) + sum(lf, n);
      }
  }
  checksum += oracle_cell_self_integral(1.0, 1.0, 1.0) + oracle_cell_self_integral(0.5, 2.0, 1.25);
  checksum += oracle_num_threads();

  oracle_cfg per = {{4, 3, 5}, {6, 4, 5}, {1.0, 0.75, 1.25}, {-1.0, -2.0, -0.5}, {1.5, 2.0, 0.5}, 1.0, 0, 0};
  oracle_cfg iso = {{3, 4, 2}, {4, 5, 3}, {0.75, 1.0, 0.5}, {-1.0, -1.5, -0.5}, {1.0, 1.5, 0.75}, 1.0, 1, 0};
  exercise(&per, &checksum);
  exercise(&iso, &checksum);
  printf("checksum %.17g\n", checksum);
  return isfinite(checksum) ? 0 : 1;
}
