/*
 * Oracle (test infrastructure only): ionization update and the Gamma <-> x
 * iteration.
 *
 * Eq. chem_ode, dx/dt = (1 - x)(Gamma + n_e C_H) - x n_e alpha_H, is
 * integrated with the time-averaged method the paper adopts from C2-Ray
 * (Sec. "Time integration"): for fixed Gamma and n_e the equation is linear
 * in x, with
 *     t_i  = 1 / (Gamma + n_e alpha)
 *     x_eq = Gamma t_i
 *     x(dt)  = x_eq + (x0 - x_eq) exp(-dt / t_i)
 *     x_avg  = x_eq + (x0 - x_eq) (t_i / dt) (1 - exp(-dt / t_i)),
 * and n_e = x_avg n_H is iterated per cell.  Readings: hydrogen only and
 * n_e = x n_H (the printed "n_e = x n_HI" is garbled); C_H = 0; alpha is the
 * case-B coefficient times the clumping factor.
 *
 * Sec. "Iterative nonlinear solve": fix x to compute Gamma, fix Gamma to
 * update x, iterate to convergence.  Reading: the tracer sees the
 * time-averaged x_avg, as in C2-Ray.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static void chem_cell(double G, double n_H, double x0, double dt, double alpha,
                      double guess, double* x_new, double* x_avg) {
  double xav = guess, xn = x0;
  for (int it = 0; it < 200; ++it) {
    const double n_e = xav * n_H;
    const double rate = G + n_e * alpha; /* 1 / t_i */
    double xend, xmean;
    if (rate > 0.0) {
      const double t_i = 1.0 / rate;
      const double x_eq = G * t_i;
      const double u = dt / t_i;
      const double e = exp(-u);
      xend = x_eq + (x0 - x_eq) * e;
      xmean = x_eq + (x0 - x_eq) * ((-expm1(-u)) / u);
    } else {
      xend = x0;
      xmean = x0;
    }
    const double change = fabs(xmean - xav);
    xav = xmean;
    xn = xend;
    if (change <= 1e-12) break;
  }
  *x_new = xn;
  *x_avg = xav;
}

void orc_chem_update(int64_t ncell, const double* gamma, const double* n_H, const double* x0,
                     double dt, double alpha, const double* x_avg_guess, double* x_new,
                     double* x_avg) {
  for (int64_t c = 0; c < ncell; ++c)
    chem_cell(gamma[c], n_H[c], x0[c], dt, alpha, x_avg_guess[c], &x_new[c], &x_avg[c]);
}

int orc_rt_step(const orc_params* p, const double* n_H, double* x, int64_t m,
                const double* pos, const double* ndot, double dt, double alpha, double tol,
                double conv_frac, int max_iter, int nthreads, double* gamma, orc_budget* b,
                int* iters) {
  if (!p || p->n < 1 || !(dt > 0.0) || max_iter < 1) return 1;
  const int64_t n = p->n, ncell = n * n * n;
  double* xav = (double*)malloc((size_t)ncell * sizeof(double));
  double* xav2 = (double*)malloc((size_t)ncell * sizeof(double));
  double* xnew = (double*)malloc((size_t)ncell * sizeof(double));
  int rc = 0, it = 0;
  if (!xav || !xav2 || !xnew) {
    rc = 2;
    goto out;
  }
  memcpy(xav, x, (size_t)ncell * sizeof(double));
  for (it = 1; it <= max_iter; ++it) {
    rc = orc_trace(p, n_H, xav, m, pos, ndot, nthreads, gamma, b);
    if (rc) goto out;
    orc_chem_update(ncell, gamma, n_H, x, dt, alpha, xav, xnew, xav2);
    int64_t changed = 0; /* cells whose step average moved by tol or more */
    for (int64_t c = 0; c < ncell; ++c)
      if (fabs(xav2[c] - xav[c]) >= tol) ++changed;
    memcpy(xav, xav2, (size_t)ncell * sizeof(double));
    if ((double)changed <= conv_frac * (double)ncell) break;
  }
  if (it > max_iter) it = max_iter;
  memcpy(x, xnew, (size_t)ncell * sizeof(double));
out:
  if (iters) *iters = it;
  free(xav);
  free(xav2);
  free(xnew);
  return rc;
}
