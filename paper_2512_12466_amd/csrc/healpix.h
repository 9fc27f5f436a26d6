// HEALPix nested pixel centres (Gorski et al. 2005), the pixelisation along
// which the paper's rays split (Sec. "Adaptive ray tracing", Fig. raysplit).
// The geometry is shared by the host, where the context fills its direction
// table with the C library's sincos, and the march, which evaluates levels
// past the table with the device's cos and sin.
//
// pix = face * Ns^2 + ipf with the in-face coordinates interleaved in ipf
// (ix on even bits, iy on odd bits); ring jr = (face/4 + 2) Ns - ix - iy - 1;
// cap rings have 1 - |z| = nr^2 / (3 Ns^2), belt rings z = (4Ns - 2jr)/(3Ns);
// phi = (pi/4) (jpll nr + ix - iy) / nr.  The azimuth is evaluated in
// [0, pi/4] and unfolded with exact swaps and sign changes, so mirror-image
// pixels have exactly mirrored vectors; every step uses correctly rounded
// FP64 operations except cos/sin.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace nrt {

__host__ __device__ inline uint32_t hp_compact(uint32_t v) {
  v &= 0x55555555u;
  v = (v | (v >> 1)) & 0x33333333u;
  v = (v | (v >> 2)) & 0x0F0F0F0Fu;
  v = (v | (v >> 4)) & 0x00FF00FFu;
  v = (v | (v >> 8)) & 0x0000FFFFu;
  return v;
}

// Pixel geometry without the trigonometry: z, sin(theta), and the azimuth
// folded into [0, pi/4] as ang = pi k / (4 nr) with the unfolding rule.
struct HpAngle {
  double z, st;
  double ang;  // folded azimuth (used when fold >= 2)
  int quad;    // quadrant of the azimuth
  int fold;    // 0: (c, s) = (1, 0); 1: c = s = sqrt(1/2); 2: (cos, sin) of ang; 3: swapped
};

// level <= 14, pix < 12 * 4^level: every integer below fits 32 bits
__host__ __device__ inline HpAngle healpix_angle(int level, uint32_t pix) {
  const int ns = 1 << level;
  const uint32_t face = pix >> (2 * level);
  const uint32_t ipf = pix - (face << (2 * level));
  const int ix = int(hp_compact(ipf));
  const int iy = int(hp_compact(ipf >> 1));
  const int row = int(face >> 2);  // 0 north, 1 equatorial, 2 south
  const int jr = (row + 2) * ns - ix - iy - 1;

  HpAngle a;
  int nr;
  if (jr < ns) {
    nr = jr;
    const double t = double(nr * nr) / double(3 * ns * ns);
    a.z = 1.0 - t;
    a.st = sqrt(t * (2.0 - t));
  } else if (jr > 3 * ns) {
    nr = 4 * ns - jr;
    const double t = double(nr * nr) / double(3 * ns * ns);
    a.z = t - 1.0;
    a.st = sqrt(t * (2.0 - t));
  } else {
    nr = ns;
    a.z = double(4 * ns - 2 * jr) / double(3 * ns);
    a.st = sqrt((1.0 - a.z) * (1.0 + a.z));
  }

  const int jpll = 2 * int(face & 3u) + (row == 1 ? 0 : 1);
  int num = jpll * nr + ix - iy;  // phi = (pi/2) num / (2 nr)
  if (num < 0) num += 8 * nr;
  if (num >= 8 * nr) num -= 8 * nr;
  a.quad = int(num >= 2 * nr) + int(num >= 4 * nr) + int(num >= 6 * nr);
  const int rem = num - a.quad * 2 * nr;
  // azimuth within the quadrant folded into [0, pi/4]: one cos and one sin,
  // swapped for the upper half
  a.ang = 0.0;
  if (rem == 0) {
    a.fold = 0;
  } else if (rem == nr) {
    a.fold = 1;
  } else {
    const bool low = rem < nr;
    const int k = low ? rem : 2 * nr - rem;
    a.ang = (3.14159265358979323846 * double(k)) / double(4 * nr);
    a.fold = low ? 2 : 3;
  }
  return a;
}

// The unit vector from the geometry and cos / sin of the folded azimuth.
__host__ __device__ inline void healpix_vector(const HpAngle& a, double ca, double sa, double& dx,
                                               double& dy, double& dz) {
  double c, s;
  if (a.fold == 0) {
    c = 1.0;
    s = 0.0;
  } else if (a.fold == 1) {
    c = 0.70710678118654752440;  // sqrt(1/2), correctly rounded
    s = c;
  } else {
    c = a.fold == 2 ? ca : sa;
    s = a.fold == 2 ? sa : ca;
  }
  double cx, sy;
  if (a.quad == 0) {
    cx = c;
    sy = s;
  } else if (a.quad == 1) {
    cx = -s;
    sy = c;
  } else if (a.quad == 2) {
    cx = -c;
    sy = -s;
  } else {
    cx = s;
    sy = -c;
  }
  dx = a.st * cx;
  dy = a.st * sy;
  dz = a.z;
}

// Pixel centre with the device's cos and sin (the march, for levels past
// the context's direction table).
__device__ inline void healpix_dir(int level, uint32_t pix, double& dx, double& dy, double& dz) {
  const HpAngle a = healpix_angle(level, pix);
  double ca = 1.0, sa = 0.0;
  if (a.fold >= 2) {
    ca = cos(a.ang);
    sa = sin(a.ang);
  }
  healpix_vector(a, ca, sa, dx, dy, dz);
}

}  // namespace nrt
