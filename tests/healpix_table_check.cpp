// Host check (test infrastructure): the context's direction table, as the
// library computes it on the host (the pixelisation's geometry from
// healpix.h, the C library's sincos), equals the oracle's directions bit for
// bit at levels 0..10.  Built and run by tests/test_healpix_table.py.
#include <cmath>
#include <cstdio>
#include "healpix.h"
extern "C" void orc_pix2vec_nest(int level, uint64_t pix, double v[3]);
int main() {  // levels 0..10: the table of every workload (l_max <= 11)
  long bad = 0, tot = 0;
  for (int l = 0; l <= 10; ++l) {
    const long npix = 12L << (2 * l);
    for (long p = 0; p < npix; ++p) {
      const nrt::HpAngle a = nrt::healpix_angle(l, uint32_t(p));
      double ca = 1.0, sa = 0.0;
      if (a.fold >= 2) ::sincos(a.ang, &sa, &ca);
      double d[3], v[3];
      nrt::healpix_vector(a, ca, sa, d[0], d[1], d[2]);
      orc_pix2vec_nest(l, p, v);
      for (int k = 0; k < 3; ++k) bad += d[k] != v[k];
      tot += 3;
    }
  }
  printf("mismatches %ld of %ld\n", bad, tot);
  return bad != 0;
}
