/*
 * Oracle (test infrastructure only): HEALPix nested pixel centres.
 *
 * The paper casts 12 level-0 rays per source and splits a ray into the 4
 * nested sub-pixels of its HEALPix pixel (Sec. "Adaptive ray tracing",
 * Fig. raysplit).  The pixelisation itself is the one of Gorski et al. 2005,
 * which the paper cites; this file writes it out from that definition:
 *
 *   nested index  pix = face * Ns^2 + ipf, ipf interleaves the bits of the
 *                 in-face coordinates (ix on even bits, iy on odd bits);
 *   ring number   jr = jrll[face] * Ns - ix - iy - 1   (1 .. 4Ns-1);
 *   polar caps    1 - z = nr^2 / (3 Ns^2),  nr = jr (north) or 4Ns - jr;
 *   equator belt  z = (4Ns - 2 jr) / (3 Ns),  nr = Ns;
 *   azimuth       phi = (pi / 4) * (jpll[face] * nr + ix - iy) / nr.
 *
 * Reading taken (the paper is silent): a ray's direction is the unit vector
 * to its pixel centre.  The azimuth is evaluated in [0, pi/4] and mapped to
 * the full circle by exact swaps and sign flips, so that mirror-image pixels
 * get exactly mirrored vectors and the pi/4 and pi/2 directions are exact.
 */
#include <math.h>
#include <stdint.h>

#include "oracle.h"

static const int64_t k_jrll[12] = {2, 2, 2, 2, 3, 3, 3, 3, 4, 4, 4, 4};
static const int64_t k_jpll[12] = {1, 3, 5, 7, 0, 2, 4, 6, 1, 3, 5, 7};

void orc_pix2vec_nest(int level, uint64_t pix, double v[3]) {
  const int64_t ns = (int64_t)1 << level;
  const uint64_t npface = (uint64_t)ns * (uint64_t)ns;
  const int64_t face = (int64_t)(pix / npface);
  const uint64_t ipf = pix % npface;

  /* de-interleave the in-face coordinates */
  int64_t ix = 0, iy = 0;
  for (int bit = 0; bit < level; ++bit) {
    ix |= (int64_t)((ipf >> (2 * bit)) & 1u) << bit;
    iy |= (int64_t)((ipf >> (2 * bit + 1)) & 1u) << bit;
  }

  const int64_t jr = k_jrll[face] * ns - ix - iy - 1;
  int64_t nr;
  double z, sin_theta;
  if (jr < ns) { /* north polar cap */
    nr = jr;
    const double t = (double)(nr * nr) / (double)(3 * ns * ns); /* 1 - z */
    z = 1.0 - t;
    sin_theta = sqrt(t * (2.0 - t));
  } else if (jr > 3 * ns) { /* south polar cap */
    nr = 4 * ns - jr;
    const double t = (double)(nr * nr) / (double)(3 * ns * ns); /* 1 + z */
    z = t - 1.0;
    sin_theta = sqrt(t * (2.0 - t));
  } else { /* equatorial belt */
    nr = ns;
    z = (double)(4 * ns - 2 * jr) / (double)(3 * ns);
    sin_theta = sqrt((1.0 - z) * (1.0 + z));
  }

  /* phi = (pi/2) * num / (2 nr), num in [0, 8 nr) */
  int64_t num = k_jpll[face] * nr + ix - iy;
  if (num < 0) num += 8 * nr;
  if (num >= 8 * nr) num -= 8 * nr;
  const int64_t quadrant = num / (2 * nr);
  const int64_t rem = num - quadrant * 2 * nr; /* angle pi*rem/(4nr) in [0,pi/2) */

  double c, s; /* cos, sin of the angle within the quadrant */
  if (rem == 0) {
    c = 1.0;
    s = 0.0;
  } else if (rem == nr) { /* exactly pi/4 */
    c = sqrt(0.5);
    s = c;
  } else if (rem < nr) {
    const double ang = (M_PI * (double)rem) / (double)(4 * nr);
    sincos(ang, &s, &c); /* the C library's joint sine and cosine */
  } else { /* pi/2 - ang with ang in (0, pi/4) */
    const double ang = (M_PI * (double)(2 * nr - rem)) / (double)(4 * nr);
    sincos(ang, &c, &s);
  }

  double cx, sy;
  switch (quadrant) {
    case 0: cx = c;  sy = s;  break;
    case 1: cx = -s; sy = c;  break;
    case 2: cx = -c; sy = -s; break;
    default: cx = s; sy = -c; break;
  }
  v[0] = sin_theta * cx;
  v[1] = sin_theta * sy;
  v[2] = z;
}
