/*
 * Oracle (test infrastructure only): frequency integrals of Eq. lut_eqn for
 * a polychromatic source, by direct quadrature over frequency.
 */
#ifndef NYXRT_ORACLE_SPECTRUM_H
#define NYXRT_ORACLE_SPECTRUM_H

#include <stdint.h>

/* Composite Gauss-Legendre rule over u = nu / nu_0 in [1, u_max], with the
   normalised photon spectrum folded into the weights:
     F(tau)       = sum_i wphi[i] exp(-tau s[i])
     G(tau)       = sum_i wphi[i] s[i] exp(-tau s[i])
     D(tau, dtau) = sum_i wphi[i] exp(-tau s[i]) (1 - exp(-dtau s[i]))
   with s[i] = sigma(u_i) / sigma_0 = u_i^-3.  kind == ORC_SPEC_MONO has no
   nodes and uses the closed forms. */
typedef struct {
  int32_t kind;
  double param;
  int64_t count;
  double* s;
  double* wphi;
} orc_spectrum;

/* Returns 0 on success, nonzero on a bad kind or parameter, or when the
   spectrum is too hard for a bounded frequency range. */
int orc_spectrum_init(orc_spectrum* sp, int32_t kind, double param);
void orc_spectrum_free(orc_spectrum* sp);

double orc_spectrum_F(const orc_spectrum* sp, double tau);
double orc_spectrum_G(const orc_spectrum* sp, double tau);
double orc_spectrum_D(const orc_spectrum* sp, double tau, double dtau);

#endif
