// Ionization update of a radiation step (Secs. "Time integration" and
// "Iterative nonlinear solve") and the Gamma <-> x iteration around the trace.
//
// For fixed Gamma and n_e, Eq. chem_ode with C_H = 0 is linear in x:
//   t_i = 1 / (Gamma + n_e alpha),  x_eq = Gamma t_i,
//   x(dt)  = x_eq + (x0 - x_eq) exp(-dt / t_i),
//   x_avg  = x_eq + (x0 - x_eq) (1 - exp(-u)) / u,  u = dt / t_i,
// and n_e = x_avg n_H is iterated per cell (C2-Ray's time averaging).  The
// tracer sees a = (1 - x_avg) n_H.
#include "internal.h"

namespace nrt {
namespace {

__global__ void k_chem(const double* __restrict__ gamma, const double* __restrict__ n_H,
                       const double* __restrict__ x0, double dt, double alpha, double tol,
                       int64_t ncell, double* x_avg, double* x_new,
                       unsigned long long* changed, const unsigned long long* skip) {
  if (skip && *skip) return;
  unsigned long long local = 0;
  for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < ncell;
       c += int64_t(gridDim.x) * blockDim.x) {
    const double G = gamma[c], nh = n_H[c], xs = x0[c];
    const double guess = x_avg[c];
    double xav = guess, xend = xs;
    for (int it = 0; it < 200; ++it) {
      const double rate = G + (xav * nh) * alpha;
      double e_end, e_mean;
      if (rate > 0.0) {
        const double t_i = 1.0 / rate;
        const double x_eq = G * t_i;
        const double u = dt / t_i;
        e_end = x_eq + (xs - x_eq) * exp(-u);
        e_mean = x_eq + (xs - x_eq) * ((-expm1(-u)) / u);
      } else {
        e_end = xs;
        e_mean = xs;
      }
      const double change = fabs(e_mean - xav);
      xav = e_mean;
      xend = e_end;
      if (change <= 1e-12) break;
    }
    x_avg[c] = xav;
    x_new[c] = xend;
    if (fabs(xav - guess) >= tol) ++local;
  }
  for (int off = 32; off > 0; off >>= 1) local += __shfl_xor(local, off);
  if (__lane_id() == 0 && local) atomicAdd(changed, local);
}

__global__ void k_copy(const double* __restrict__ src, double* dst, int64_t count) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
       i += int64_t(gridDim.x) * blockDim.x)
    dst[i] = src[i];
}

}  // namespace

hipError_t launch_chem(const nrt_ctx* c, const double* gamma, double dt, double alpha, double tol,
                       double* x_avg, double* x_new, hipStream_t s,
                       const unsigned long long* skip) {
  int64_t blocks = (c->lay.cells + 255) / 256;
  if (blocks > int64_t(c->cu_count) * 16) blocks = int64_t(c->cu_count) * 16;
  hipLaunchKernelGGL(k_chem, dim3(unsigned(blocks)), dim3(256), 0, s, gamma, c->n_H, c->x, dt,
                     alpha, tol, c->lay.cells, x_avg, x_new, &c->acc->chem_changed, skip);
  return hipGetLastError();
}

hipError_t launch_copy(const nrt_ctx* c, const double* src, double* dst) {
  int64_t blocks = (c->lay.cells + 255) / 256;
  if (blocks > int64_t(c->cu_count) * 16) blocks = int64_t(c->cu_count) * 16;
  hipLaunchKernelGGL(k_copy, dim3(unsigned(blocks)), dim3(256), 0, c->stream, src, dst,
                     c->lay.cells);
  return hipGetLastError();
}

}  // namespace nrt
