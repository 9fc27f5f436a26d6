/*
 * Sanitizer test program for the oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Built twice by tests/test_oracle_sanitizers.py with gcc (never for a GPU):
 * with AddressSanitizer + UndefinedBehaviorSanitizer, and with
 * ThreadSanitizer for the threaded trace.  It runs every entry point of the
 * oracle on small deterministic inputs (a fixed linear congruential
 * generator, no files) and checks the photon budget identity of each trace,
 * so that the sanitizers see the code paths the tests use: both boundaries,
 * every correction mode, a spectrum, injected rays with the segment log,
 * source merging and a radiation step.  Exit status 0 when every check holds.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static uint64_t lcg = 0x2512124660000001ull;
static double uniform(void) {
  lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
  return (double)(lcg >> 11) * (1.0 / 9007199254740992.0);
}

static int check_budget(const char* what, const orc_budget* b) {
  const double err = fabs(b->absorbed + b->escaped + b->truncated - b->emitted);
  if (!(err <= 1e-12 * b->emitted) || b->segments == 0) {
    fprintf(stderr, "%s: budget error %g of %g, %llu segments\n", what, err, b->emitted,
            (unsigned long long)b->segments);
    return 1;
  }
  return 0;
}

int main(void) {
  const int n = 12;
  const int64_t ncell = (int64_t)n * n * n;
  double* n_H = malloc(sizeof(double) * ncell);
  double* x = malloc(sizeof(double) * ncell);
  double* gamma = malloc(sizeof(double) * ncell);
  if (!n_H || !x || !gamma) return 2;
  for (int64_t c = 0; c < ncell; ++c) {
    n_H[c] = 1e-3 * exp(uniform() - 0.5);
    x[c] = uniform() < 0.3 ? 1.0 - 1e-4 : 0.0;
  }
  enum { M = 5 };
  double pos[3 * M], ndot[M];
  for (int k = 0; k < M; ++k) {
    for (int a = 0; a < 3; ++a) pos[3 * k + a] = uniform() * n;
    ndot[k] = 1e50 * (0.5 + uniform());
  }
  int bad = 0;
  orc_budget b;
  for (int periodic = 0; periodic <= 1; ++periodic) {
    for (int corr = 0; corr <= ORC_CORR_NAIVE; ++corr) {
      orc_params p = {n, 4.0e20, periodic, 6.30e-18, 4.0, 5, 30.0, 4e-4, corr,
                      ORC_SPEC_MONO, 0.0};
      if (orc_trace(&p, n_H, x, M, pos, ndot, 4, gamma, &b)) return 3;
      char what[64];
      snprintf(what, sizeof what, "trace periodic %d corr %d", periodic, corr);
      bad |= check_budget(what, &b);
    }
  }
  orc_params ps = {n, 4.0e20, 1, 6.30e-18, 4.0, 4, 30.0, 4e-4, ORC_CORR_CONSERVATIVE,
                   ORC_SPEC_BLACKBODY, 5e4};
  if (orc_trace(&ps, n_H, x, M, pos, ndot, 3, gamma, &b)) return 4;
  bad |= check_budget("trace blackbody", &b);

  /* injected rays with the segment log */
  enum { K = 40 };
  double org[3 * K], dir[3 * K], L[K];
  int32_t lev[K];
  for (int r = 0; r < K; ++r) {
    double d2 = 0.0;
    for (int a = 0; a < 3; ++a) {
      org[3 * r + a] = uniform() * n;
      dir[3 * r + a] = uniform() - 0.5;
      d2 += dir[3 * r + a] * dir[3 * r + a];
    }
    for (int a = 0; a < 3; ++a) dir[3 * r + a] /= sqrt(d2);
    lev[r] = r % 6;
    L[r] = 1e45;
  }
  orc_params pi = {n, 4.0e20, 0, 6.30e-18, 0.0, 7, 30.0, 4e-4, ORC_CORR_CONSERVATIVE,
                   ORC_SPEC_MONO, 0.0};
  int64_t cell[256], ijk[3 * 256], nlog = 0;
  double ds[256];
  if (orc_trace_rays(&pi, n_H, x, K, org, dir, lev, L, gamma, &b, 256, cell, ds, ijk, &nlog))
    return 5;
  bad |= check_budget("injected rays", &b);

  /* spectrum integrals */
  double tau[4] = {0.0, 0.5, 5.0, 50.0}, dt[4] = {0.1, 1.0, 0.0, 2.0}, F[4], D[4], G[4];
  if (orc_spectrum_eval(ORC_SPEC_POWERLAW, 4.0, 4, tau, dt, F, D, G)) return 6;

  /* merging: clustered cell-centred sources in ionized bubbles */
  enum { S = 64 };
  double sp[3 * S], sf[S];
  for (int k = 0; k < S; ++k) {
    for (int a = 0; a < 3; ++a) sp[3 * k + a] = floor(uniform() * 4.0) + 4.5;
    sf[k] = 1e49;
  }
  double* xb = malloc(sizeof(double) * ncell);
  if (!xb) return 2;
  for (int64_t c = 0; c < ncell; ++c) xb[c] = 1.0 - 1e-4;
  orc_merge_params mp = {2.0, 0.9, 0.9, 8, 8.0, 1.0, 1e-6, 2};
  int32_t cells[3 * S];
  double flux[S], radius[S];
  const int64_t m2 = orc_merge_sources(&mp, n, 1, xb, S, sp, sf, cells, flux, radius);
  if (m2 < 1) return 7;
  double total = 0.0;
  for (int64_t k = 0; k < m2; ++k) total += flux[k];
  if (fabs(total - S * 1e49) > 1e-12 * S * 1e49) {
    fprintf(stderr, "merge: flux %g of %g\n", total, S * 1e49);
    bad = 1;
  }

  /* one radiation step */
  orc_params pr = {n, 2.0e20, 0, 6.30e-18, 4.0, 5, 30.0, 1e-5, ORC_CORR_CONSERVATIVE,
                   ORC_SPEC_MONO, 0.0};
  for (int64_t c = 0; c < ncell; ++c) xb[c] = 0.0;
  int iters = 0;
  double src[3] = {6.5, 6.5, 6.5}, rate[1] = {5e48};
  if (orc_rt_step(&pr, n_H, xb, 1, src, rate, 3.15576e13, 2.59e-13, 1e-6, 0.0, 50, 2, gamma, &b,
                  &iters))
    return 8;
  bad |= check_budget("radiation step", &b);
  free(xb);
  free(n_H);
  free(x);
  free(gamma);
  if (!bad) printf("sanitized oracle run: ok\n");
  return bad;
}
