/*
 * Oracle (test infrastructure only): the frequency integral of Eq. lut_eqn
 * for a polychromatic source, evaluated by plain quadrature.
 *
 * Eq. lut_eqn integrates L_nu e^{-tau_nu} (1 - e^{-dtau_nu}) / (h nu) over
 * nu >= nu_0.  Writing u = nu / nu_0, the photon rate of a ray splits as
 * L phi(u) du with a normalised photon spectrum phi (int_1^inf phi du = 1),
 * and the optical depths scale with the cross-section: tau_nu = tau_0 s(u),
 * s(u) = sigma_nu / sigma_0.  The paper tabulates the integral in the
 * threshold optical depth tau_0 following C2-Ray (Sec. "Flux computation")
 * and gives neither the spectrum nor sigma_nu; the readings taken here are
 *   - s(u) = u^-3 (the hydrogenic power law of the threshold cross-section);
 *   - spectra: a blackbody at temperature T, phi ~ u^2 / (e^{beta u} - 1)
 *     with beta = 13.6 eV / (k_B T), or a power law phi ~ u^-alpha.
 * Per unit L the ray then carries F(tau_0) = int phi e^{-tau_0 s} du photons
 * past optical depth tau_0, a cell of depth dtau_0 absorbs
 *   D(tau_0, dtau_0) = int phi e^{-tau_0 s} (1 - e^{-dtau_0 s}) du
 * = F(tau_0) - F(tau_0 + dtau_0), and the n_HI -> 0 limit of the deposit
 * (footnote on the optically thin table in Sec. "Numerical instability for
 * low n_H neighbor cells") is G(tau_0) dtau_0 with G = int phi s e^{-tau_0 s}
 * du = -F'(tau_0).
 *
 * The integrals are composite 16-point Gauss-Legendre sums over geometric
 * panels [2^{k/8}, 2^{(k+1)/8}] of u, up to the u where the remaining
 * spectrum is below 1e-20 of the total.  D is summed with expm1 so that a thin
 * cell does not cancel.
 */
#include "spectrum.h"

#include <math.h>
#include <stdlib.h>

#include "oracle.h"

#define GL_N 16
#define PANELS_PER_OCTAVE 8

/* Gauss-Legendre nodes and weights on [-1, 1]: Newton's method on the
   Legendre polynomial P_n from the Chebyshev-like initial guesses, with
   P_n and P_n' from the three-term recurrence. */
static void gauss_legendre(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (fabs(dz) < 1e-16) break;
    }
    {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
    }
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

/* 13.6 eV over Boltzmann's constant (8.617333262e-5 eV/K), in kelvin */
#define ORC_E0_OVER_KB (13.6 / 8.617333262e-5)

/* un-normalised photon spectrum at u >= 1 */
static double spectrum_phi(int32_t kind, double param, double u) {
  if (kind == ORC_SPEC_BLACKBODY) {
    const double beta = ORC_E0_OVER_KB / param;
    return u * u / expm1(beta * u);
  }
  return pow(u, -param); /* ORC_SPEC_POWERLAW */
}

/* u beyond which the spectrum holds less than ~1e-20 of its photons */
static double spectrum_umax(int32_t kind, double param) {
  if (kind == ORC_SPEC_BLACKBODY) {
    /* past U the spectrum holds about U^2 e^{-beta (U - 1)} of its photons */
    const double beta = ORC_E0_OVER_KB / param;
    double u = 2.0;
    while (beta * (u - 1.0) - 2.0 * log(u) < 50.0) u *= 2.0;
    return u;
  }
  /* power law: int_U^inf u^-a du / int_1^inf = U^{1-a} */
  return pow(1e-20, 1.0 / (1.0 - param));
}

int orc_spectrum_init(orc_spectrum* sp, int32_t kind, double param) {
  sp->kind = kind;
  sp->param = param;
  sp->count = 0;
  sp->s = sp->wphi = NULL;
  if (kind == ORC_SPEC_MONO) return 0;
  if (kind == ORC_SPEC_BLACKBODY) {
    if (!(param >= 1e3 && param <= 1e7)) return 1;
  } else if (kind == ORC_SPEC_POWERLAW) {
    if (!(param >= 2.5 && param <= 50.0)) return 1;
  } else {
    return 1;
  }
  const double umax = spectrum_umax(kind, param);
  if (!(umax <= 0x1p60)) return 1;
  const int64_t panels = (int64_t)ceil(log2(umax) * PANELS_PER_OCTAVE);
  sp->count = panels * GL_N;
  sp->s = (double*)malloc((size_t)sp->count * sizeof(double));
  sp->wphi = (double*)malloc((size_t)sp->count * sizeof(double));
  if (!sp->s || !sp->wphi) {
    orc_spectrum_free(sp);
    return 1;
  }
  double gx[GL_N], gw[GL_N];
  gauss_legendre(GL_N, gx, gw);
  double z = 0.0;
  for (int64_t k = 0; k < panels; ++k) {
    const double a = exp2((double)k / PANELS_PER_OCTAVE);
    const double b = exp2((double)(k + 1) / PANELS_PER_OCTAVE);
    for (int i = 0; i < GL_N; ++i) {
      const double u = 0.5 * (a + b) + 0.5 * (b - a) * gx[i];
      const double wphi = 0.5 * (b - a) * gw[i] * spectrum_phi(kind, param, u);
      sp->s[k * GL_N + i] = 1.0 / (u * u * u);
      sp->wphi[k * GL_N + i] = wphi;
      z += wphi;
    }
  }
  for (int64_t i = 0; i < sp->count; ++i) sp->wphi[i] /= z;
  return 0;
}

void orc_spectrum_free(orc_spectrum* sp) {
  free(sp->s);
  free(sp->wphi);
  sp->s = sp->wphi = NULL;
  sp->count = 0;
}

double orc_spectrum_F(const orc_spectrum* sp, double tau) {
  if (sp->kind == ORC_SPEC_MONO) return exp(-tau);
  double f = 0.0;
  for (int64_t i = 0; i < sp->count; ++i) f += sp->wphi[i] * exp(-tau * sp->s[i]);
  return f;
}

double orc_spectrum_G(const orc_spectrum* sp, double tau) {
  if (sp->kind == ORC_SPEC_MONO) return exp(-tau);
  double g = 0.0;
  for (int64_t i = 0; i < sp->count; ++i) g += sp->wphi[i] * sp->s[i] * exp(-tau * sp->s[i]);
  return g;
}

double orc_spectrum_D(const orc_spectrum* sp, double tau, double dtau) {
  if (sp->kind == ORC_SPEC_MONO) return exp(-tau) * (-expm1(-dtau));
  double d = 0.0;
  for (int64_t i = 0; i < sp->count; ++i)
    d += sp->wphi[i] * exp(-tau * sp->s[i]) * (-expm1(-dtau * sp->s[i]));
  return d;
}

int orc_spectrum_eval(int32_t kind, double param, int64_t k, const double* tau,
                      const double* dtau, double* F, double* D, double* G) {
  orc_spectrum sp;
  if (k < 0 || orc_spectrum_init(&sp, kind, param)) return 1;
  for (int64_t i = 0; i < k; ++i) {
    if (F) F[i] = orc_spectrum_F(&sp, tau[i]);
    if (G) G[i] = orc_spectrum_G(&sp, tau[i]);
    if (D) D[i] = orc_spectrum_D(&sp, tau[i], dtau ? dtau[i] : 0.0);
  }
  orc_spectrum_free(&sp);
  return 0;
}
