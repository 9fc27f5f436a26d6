// Polychromatic sources: the table of Phi(tau) = -ln F(tau) that the march
// uses in place of a per-frequency sum (Sec. "Flux computation": the
// frequency integral of Eq. lut_eqn is tabulated in the threshold optical
// depth, after C2-Ray).
//
// With u = nu / nu_0 and the cross-section sigma_0 u^-3, a photon at u sees
// the optical depth tau s with s = u^-3 in (0, 1].  In the variable s the
// normalised photon spectrum is psi(s) ds, and
//   F(tau) = int_0^1 psi(s) e^{-tau s} ds / int_0^1 psi(s) ds,
// a Laplace transform, so Phi = -ln F is smooth and increasing with
// Phi' = <s>_tau and Phi'' = -Var_tau(s), the mean and variance of s under
// the weight psi(s) e^{-tau s}.  Blackbody: phi(u) ~ u^2 / (e^{beta u} - 1),
// beta = 13.6 eV / kT, so psi(s) ~ u^6 / (e^{beta u} - 1); power law
// phi ~ u^-alpha gives psi ~ u^(4 - alpha).
//
// The moments at each node come from tanh-sinh quadrature over s in (0, 1)
// (s = 1 / (1 + e^{pi sinh t}), a trapezoid rule in t with step 1/256 over
// |t| <= 6.5), which resolves the integrable endpoint behaviour of psi and
// the concentration of the weight near s ~ 1/tau at large tau.  The interval
// coefficients are the quintic Hermite interpolant through Phi, Phi' and
// Phi'' at both ends; across an interval Phi rises by ln(m0_q / m0_{q+1}),
// taken from the moments directly so that it carries no cancellation.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "internal.h"

namespace nrt {
namespace {

constexpr int kTsBlock = 256;
constexpr double kTsStep = 1.0 / 256.0;
constexpr int kTsHalf = 1664;  // 6.5 / kTsStep
constexpr double kPi = 3.14159265358979323846;
// 13.6 eV over Boltzmann's constant (8.617333262e-5 eV/K), in kelvin
constexpr double kE0OverKb = 13.6 / 8.617333262e-5;

__host__ __device__ inline double node_tau(int q) {
  const int e = q >> kSpecLog2Sub, m = q & (kSpecSub - 1);
  return std::ldexp(1.0 + double(m) / kSpecSub, e) - 1.0;
}

struct TsPoint {
  double s, ln_psi_w;  // abscissa, ln(psi(s) * quadrature weight)
};

// tanh-sinh point j in [-kTsHalf, kTsHalf]; ln_psi_w = -inf where the
// weight or the spectrum underflows
__device__ TsPoint ts_point(int j, int kind, double param) {
  const double t = j * kTsStep;
  const double v = kPi * sinh(t);
  const double ev = exp(-fabs(v));  // in (0, 1]
  TsPoint p;
  double ln_s;
  if (v >= 0.0) {
    p.s = ev / (1.0 + ev);
    ln_s = -v - log1p(ev);
  } else {
    p.s = 1.0 / (1.0 + ev);
    ln_s = -log1p(ev);
  }
  // ds/dt = pi cosh t s (1 - s), s (1 - s) = ev / (1 + ev)^2
  const double ln_w = log(kTsStep * kPi * cosh(t)) - fabs(v) - 2.0 * log1p(ev);
  const double ln_u = -ln_s / 3.0;
  double ln_psi;
  if (kind == NRT_SPEC_BLACKBODY) {
    const double bu = (kE0OverKb / param) * exp(ln_u);
    ln_psi = 6.0 * ln_u - bu - log(-expm1(-bu));
  } else {
    ln_psi = (4.0 - param) * ln_u;
  }
  p.ln_psi_w = ln_psi + ln_w;
  return p;
}

__device__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int h = kTsBlock / 2; h > 0; h >>= 1) {
    if (int(threadIdx.x) < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// one block per node: m0 = int psi e^{-tau s}, mean and variance of s
__global__ __launch_bounds__(kTsBlock) void k_spec_nodes(int kind, double param, double* m0,
                                                         double* mean, double* var) {
  __shared__ double red[kTsBlock];
  const int q = blockIdx.x;
  const double tau = node_tau(q);
  double a0 = 0.0, a1 = 0.0;
  for (int j = -kTsHalf + int(threadIdx.x); j <= kTsHalf; j += kTsBlock) {
    const TsPoint p = ts_point(j, kind, param);
    const double f = exp(p.ln_psi_w - tau * p.s);
    a0 += f;
    a1 += f * p.s;
  }
  const double s0 = block_sum(a0, red);
  const double s1 = block_sum(a1, red);
  const double mu = s0 > 0.0 ? s1 / s0 : 0.0;
  double a2 = 0.0;
  for (int j = -kTsHalf + int(threadIdx.x); j <= kTsHalf; j += kTsBlock) {
    const TsPoint p = ts_point(j, kind, param);
    const double f = exp(p.ln_psi_w - tau * p.s);
    a2 += f * (p.s - mu) * (p.s - mu);
  }
  const double s2 = block_sum(a2, red);
  if (threadIdx.x == 0) {
    m0[q] = s0;
    mean[q] = mu;
    var[q] = s0 > 0.0 ? s2 / s0 : 0.0;
  }
}

// interval q: quintic Hermite coefficients in x = (tau - tau_q) / W_q
__global__ void k_spec_coef(int nint, const double* m0, const double* mean, const double* var,
                            SpecRec64* r64, SpecRec32* r32) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nint) return;
  const double w = ldexp(1.0, (q >> kSpecLog2Sub) - kSpecLog2Sub);
  const double f0 = -log(m0[q] / m0[0]);
  const double rise = log(m0[q] / m0[q + 1]);  // Phi_{q+1} - Phi_q
  const double d0 = w * mean[q], d1 = w * mean[q + 1];
  const double s0 = -w * w * var[q], s1 = -w * w * var[q + 1];
  // p(1) = f0 + rise, p'(1) = d1, p''(1) = s1
  const double A = rise - d0 - 0.5 * s0, B = d1 - d0 - s0, C = s1 - s0;
  double c[6];
  c[0] = f0;
  c[1] = d0;
  c[2] = 0.5 * s0;
  c[3] = 10.0 * A - 4.0 * B + 0.5 * C;
  c[4] = -15.0 * A + 7.0 * B - C;
  c[5] = 6.0 * A - 3.0 * B + 0.5 * C;
  SpecRec64 a;
  for (int k = 0; k < 5; ++k) a.c[k] = c[k + 1];
  a.c[5] = c[0];
  a.c[6] = a.c[7] = 0.0;
  r64[q] = a;
  SpecRec32 b;
  for (int k = 0; k < 5; ++k) b.c[k] = float(c[k + 1]);
  b.c[5] = 0.0f;
  b.c0 = c[0];
  r32[q] = b;
}

}  // namespace

nrt_status build_spectrum_table(nrt_ctx* c) {
  const nrt_grid_desc& d = c->desc;
  double* m0 = c->spec_nodes;
  double* mean = m0 + kSpecNodes;
  double* var = mean + kSpecNodes;
  hipLaunchKernelGGL(k_spec_nodes, dim3(kSpecNodes), dim3(kTsBlock), 0, c->stream,
                     int(d.spectrum), d.spec_param, m0, mean, var);
  hipError_t e = hipGetLastError();
  std::vector<double> h(kSpecNodes);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h.data(), m0, kSpecNodes * sizeof(double), hipMemcpyDeviceToHost,
                       c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    c->err = std::string("spectrum table: ") + hipGetErrorString(e);
    return NRT_ERR_DEVICE;
  }
  if (!(h[0] > 0.0) || !std::isfinite(h[0])) {
    c->err = "spectrum table: the spectrum integrates to zero";
    return NRT_ERR_ARG;
  }
  // A ray stops once F <= e^{-tau_max}, so a cell starts at Phi < tau_max.
  // The table ends at the first octave boundary where Phi >= tau_max +
  // 6 ln 10: a cell that reaches past it absorbs all the ray carries, which
  // overstates its deposit by at most F(tau_end) / F(tau_in) < 1e-6.  Every
  // node before it must have a finite, positive m0.
  const double need = d.tau_max + 6.0 * std::log(10.0);
  int nint = 0;
  for (int oct = 1; oct <= kSpecMaxOctaves; ++oct) {
    const int q = oct * kSpecSub;
    bool ok = true;
    for (int k = (oct - 1) * kSpecSub; k <= q && ok; ++k)
      ok = h[k] > 0.0 && std::isfinite(h[k]);
    if (!ok) break;
    if (-std::log(h[q] / h[0]) >= need) {
      nint = q;
      break;
    }
  }
  if (nint == 0) {
    c->err = "spectrum too hard for the table: F(tau) does not fall to 1e-6 exp(-tau_max) "
             "within tau < 2^64";
    return NRT_ERR_ARG;
  }
  hipLaunchKernelGGL(k_spec_coef, dim3((nint + 255) / 256), dim3(256), 0, c->stream, nint, m0,
                     mean, var, c->spec64, c->spec32);
  e = hipGetLastError();
  if (e != hipSuccess) {
    c->err = std::string("spectrum table: ") + hipGetErrorString(e);
    return NRT_ERR_DEVICE;
  }
  c->spec_nint = nint;
  return NRT_OK;
}

}  // namespace nrt
