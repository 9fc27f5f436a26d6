/*
 * Oracle (test infrastructure only): source merging, Sec. "Source Merging
 * Algorithm" and Alg. source_merge.
 *
 *   dedupe     sources that fall in the same grid cell are merged by summing
 *              their rates; the list is sorted (Sec. "Source Merging
 *              Algorithm", first paragraph after the related-work survey).
 *   max_radius shells r = dr, 2 dr, ... <= R_max around the source cell; a
 *              shell passes if N_ion / N_tot >= f_req, or, when
 *              N_tot < N_min, if every sample is ionized; the radius is the
 *              last passing shell (0 if the source cell itself is not
 *              ionized, R_max if every shell passes).
 *   merge      pairs with min-image d^2 <= (f_ov (r_a + r_b))^2 + eps and
 *              r_a, r_b > 0 are united (union-find); each group becomes one
 *              source with the summed rate, the largest radius, and the
 *              flux-weighted centroid (periodic unwrap), rounded, wrapped and
 *              snapped to the nearest member cell; the result is sorted
 *              lexicographically.
 *
 * Readings where the paper is silent:
 *   - cell of a source = floor of its position; the sort key is (i, j, k)
 *     with i most significant; equal cells sum rates in input order.
 *   - the "checked point samples" of a shell are the distinct cells hit by
 *     floor(centre + r d_k) over the HEALPix pixel centres d_k of level
 *     shell_level, centre = cell index + 1/2 (wrapped if periodic, dropped
 *     if outside a non-periodic box).  Shell radii are r = k dr.
 *   - the text's d^2 <= r_sum^2 + eps is used (the listing omits eps).
 *   - the centroid is computed on cell indices, unwrapped to the minimum
 *     image of each member relative to the group's lowest-sorted member,
 *     rounded with floor(c + 1/2); the snap picks the member with the
 *     smallest min-image squared distance, ties to the lowest-sorted one.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

typedef struct {
  int64_t key, idx;
  double flux;
} keyed;

static int cmp_keyed(const void* pa, const void* pb) {
  const keyed* a = (const keyed*)pa;
  const keyed* b = (const keyed*)pb;
  if (a->key != b->key) return a->key < b->key ? -1 : 1;
  if (a->idx != b->idx) return a->idx < b->idx ? -1 : 1;
  return 0;
}

static int64_t wrapi(int64_t i, int64_t n) { return ((i % n) + n) % n; }

/* minimum-image difference of two cell coordinates */
static int64_t min_image(int64_t d, int64_t n, int periodic) {
  if (!periodic) return d;
  d = wrapi(d, n);
  if (2 * d > n) d -= n;
  return d;
}

int64_t orc_dedupe_sort(int32_t n, int64_t m, const double* pos, const double* ndot,
                        int32_t* cells_out, double* flux_out) {
  if (n < 1 || m < 0) return -1;
  if (m == 0) return 0;
  keyed* k = (keyed*)malloc((size_t)m * sizeof(keyed));
  if (!k) return -2;
  for (int64_t s = 0; s < m; ++s) {
    int64_t c[3];
    for (int ax = 0; ax < 3; ++ax) {
      const double q = pos[3 * s + ax];
      if (!(q >= 0.0 && q < (double)n)) {
        free(k);
        return -1;
      }
      c[ax] = (int64_t)floor(q);
    }
    k[s].key = (c[0] * n + c[1]) * n + c[2];
    k[s].idx = s;
    k[s].flux = ndot[s];
  }
  qsort(k, (size_t)m, sizeof(keyed), cmp_keyed);
  int64_t out = 0;
  for (int64_t s = 0; s < m; ++s) {
    if (out > 0 && s > 0 && k[s].key == k[s - 1].key) {
      flux_out[out - 1] += k[s].flux;
      continue;
    }
    const int64_t key = k[s].key;
    cells_out[3 * out + 0] = (int32_t)(key / ((int64_t)n * n));
    cells_out[3 * out + 1] = (int32_t)((key / n) % n);
    cells_out[3 * out + 2] = (int32_t)(key % n);
    flux_out[out] = k[s].flux;
    ++out;
  }
  free(k);
  return out;
}

static int cmp_i64(const void* pa, const void* pb) {
  const int64_t a = *(const int64_t*)pa, b = *(const int64_t*)pb;
  return a < b ? -1 : (a > b ? 1 : 0);
}

int orc_max_radius(const orc_merge_params* mp, int32_t n, int32_t periodic, const double* x,
                   int64_t m, const int32_t* cells, double* radius_out) {
  if (!mp || n < 1 || m < 0 || !(mp->dr > 0.0) || mp->shell_level < 0 ||
      mp->shell_level > 10)
    return 1;
  const int64_t nn = n;
  const int64_t nsamp = 12 * ((int64_t)1 << (2 * mp->shell_level));
  double* dirs = (double*)malloc((size_t)nsamp * 3 * sizeof(double));
  int64_t* hit = (int64_t*)malloc((size_t)nsamp * sizeof(int64_t));
  if (!dirs || !hit) {
    free(dirs);
    free(hit);
    return 2;
  }
  for (int64_t q = 0; q < nsamp; ++q) orc_pix2vec_nest(mp->shell_level, (uint64_t)q, dirs + 3 * q);

  for (int64_t s = 0; s < m; ++s) {
    const int64_t ci = cells[3 * s], cj = cells[3 * s + 1], ck = cells[3 * s + 2];
    if (x[ci + nn * (cj + nn * ck)] < mp->x_th) {
      radius_out[s] = 0.0;
      continue;
    }
    double result = mp->r_max;
    for (int64_t kk = 1;; ++kk) {
      const double r = (double)kk * mp->dr;
      if (!(r <= mp->r_max)) break;
      int64_t nh = 0;
      for (int64_t q = 0; q < nsamp; ++q) {
        int64_t c[3];
        const int64_t base[3] = {ci, cj, ck};
        int ok = 1;
        for (int ax = 0; ax < 3; ++ax) {
          const double pa = ((double)base[ax] + 0.5) + r * dirs[3 * q + ax];
          int64_t v = (int64_t)floor(pa);
          if (periodic)
            v = wrapi(v, nn);
          else if (v < 0 || v >= nn)
            ok = 0;
          c[ax] = v;
        }
        if (ok) hit[nh++] = c[0] + nn * (c[1] + nn * c[2]);
      }
      qsort(hit, (size_t)nh, sizeof(int64_t), cmp_i64);
      int64_t ntot = 0, nion = 0;
      for (int64_t q = 0; q < nh; ++q) {
        if (q > 0 && hit[q] == hit[q - 1]) continue;
        ++ntot;
        if (x[hit[q]] >= mp->x_th) ++nion;
      }
      int pass;
      if (ntot < mp->n_min)
        pass = (nion == ntot);
      else
        pass = !((double)nion / (double)ntot < mp->f_req);
      if (!pass) {
        result = r - mp->dr;
        break;
      }
    }
    radius_out[s] = result;
  }
  free(dirs);
  free(hit);
  return 0;
}

static int64_t uf_find(int64_t* parent, int64_t a) {
  while (parent[a] != a) {
    parent[a] = parent[parent[a]];
    a = parent[a];
  }
  return a;
}

static void uf_unite(int64_t* parent, int64_t a, int64_t b) {
  a = uf_find(parent, a);
  b = uf_find(parent, b);
  if (a == b) return;
  if (a < b)
    parent[b] = a;
  else
    parent[a] = b;
}

static int overlaps(const orc_merge_params* mp, int32_t n, int32_t periodic,
                    const int32_t* ca, const int32_t* cb, double ra, double rb) {
  if (!(ra > 0.0 && rb > 0.0)) return 0;
  double d2 = 0.0;
  for (int ax = 0; ax < 3; ++ax) {
    const double dd = (double)min_image((int64_t)ca[ax] - cb[ax], n, periodic);
    d2 += dd * dd;
  }
  const double rsum = mp->f_ov * (ra + rb);
  return d2 <= rsum * rsum + mp->eps;
}

typedef struct {
  int64_t key;
  int32_t c[3];
  double flux, radius;
} merged;

static int cmp_merged(const void* pa, const void* pb) {
  const merged* a = (const merged*)pa;
  const merged* b = (const merged*)pb;
  return a->key < b->key ? -1 : (a->key > b->key ? 1 : 0);
}

int64_t orc_merge_sources(const orc_merge_params* mp, int32_t n, int32_t periodic,
                          const double* x, int64_t m, const double* pos, const double* ndot,
                          int32_t* cells_out, double* flux_out, double* radius_out) {
  if (!mp || n < 1 || m < 0) return -1;
  if (m == 0) return 0;
  const int64_t nn = n;
  int32_t* cells = (int32_t*)malloc((size_t)m * 3 * sizeof(int32_t));
  double* flux = (double*)malloc((size_t)m * sizeof(double));
  double* rad = (double*)malloc((size_t)m * sizeof(double));
  int64_t* parent = (int64_t*)malloc((size_t)m * sizeof(int64_t));
  merged* out = (merged*)malloc((size_t)m * sizeof(merged));
  int64_t rc = -2;
  if (!cells || !flux || !rad || !parent || !out) goto done;
  const int64_t m1 = orc_dedupe_sort(n, m, pos, ndot, cells, flux);
  if (m1 < 0) {
    rc = m1;
    goto done;
  }
  if (orc_max_radius(mp, n, periodic, x, m1, cells, rad)) {
    rc = -1;
    goto done;
  }
  for (int64_t a = 0; a < m1; ++a) parent[a] = a;

  /* all pairs (a, b), a < b; pairs farther apart than 2 f_ov R_max can
     never overlap, so candidates are taken from a uniform binning whose
     bins are at least that wide (every pair within reach is visited). */
  {
    const double reach = 2.0 * mp->f_ov * mp->r_max + sqrt(mp->eps > 0 ? mp->eps : 0.0) + 1.0;
    int64_t nb = (int64_t)floor((double)nn / reach);
    if (nb < 3) nb = 1;
    if (nb == 1) {
      for (int64_t a = 0; a < m1; ++a)
        for (int64_t b = a + 1; b < m1; ++b)
          if (overlaps(mp, n, periodic, cells + 3 * a, cells + 3 * b, rad[a], rad[b]))
            uf_unite(parent, a, b);
    } else {
      /* bin of a cell coordinate: v * nb / n; bins are >= reach cells wide */
      const int64_t nbin = nb * nb * nb;
      int64_t* head = (int64_t*)malloc((size_t)nbin * sizeof(int64_t));
      int64_t* nxt = (int64_t*)malloc((size_t)m1 * sizeof(int64_t));
      if (!head || !nxt) {
        free(head);
        free(nxt);
        goto done;
      }
      for (int64_t q = 0; q < nbin; ++q) head[q] = -1;
      for (int64_t a = m1 - 1; a >= 0; --a) {
        if (!(rad[a] > 0.0)) continue;
        const int64_t bx = cells[3 * a] * nb / nn, by = cells[3 * a + 1] * nb / nn,
                      bz = cells[3 * a + 2] * nb / nn;
        const int64_t q = bx + nb * (by + nb * bz);
        nxt[a] = head[q];
        head[q] = a;
      }
      for (int64_t a = 0; a < m1; ++a) {
        if (!(rad[a] > 0.0)) continue;
        const int64_t bx = cells[3 * a] * nb / nn, by = cells[3 * a + 1] * nb / nn,
                      bz = cells[3 * a + 2] * nb / nn;
        for (int64_t dz = -1; dz <= 1; ++dz)
          for (int64_t dy = -1; dy <= 1; ++dy)
            for (int64_t dx = -1; dx <= 1; ++dx) {
              int64_t qx = bx + dx, qy = by + dy, qz = bz + dz;
              if (periodic) {
                qx = wrapi(qx, nb);
                qy = wrapi(qy, nb);
                qz = wrapi(qz, nb);
              } else if (qx < 0 || qx >= nb || qy < 0 || qy >= nb || qz < 0 || qz >= nb) {
                continue;
              }
              for (int64_t b = head[qx + nb * (qy + nb * qz)]; b >= 0; b = nxt[b])
                if (b > a &&
                    overlaps(mp, n, periodic, cells + 3 * a, cells + 3 * b, rad[a], rad[b]))
                  uf_unite(parent, a, b);
            }
      }
      free(head);
      free(nxt);
    }
  }

  /* collapse groups.  unite() hooks the larger root under the smaller, so
     every root is its group's lowest member; members are listed per root in
     increasing (sorted) order. */
  int64_t* root = parent; /* reused after full path compression */
  int64_t* first = (int64_t*)malloc((size_t)m1 * sizeof(int64_t));
  int64_t* link = (int64_t*)malloc((size_t)m1 * sizeof(int64_t));
  if (!first || !link) {
    free(first);
    free(link);
    goto done;
  }
  for (int64_t a = 0; a < m1; ++a) root[a] = uf_find(parent, a);
  for (int64_t a = 0; a < m1; ++a) first[a] = -1;
  for (int64_t b = m1 - 1; b >= 0; --b) {
    link[b] = first[root[b]];
    first[root[b]] = b;
  }
  int64_t nout = 0;
  for (int64_t a = 0; a < m1; ++a) {
    if (root[a] != a) continue;
    int64_t size = 0;
    double ftot = 0.0, rmax = 0.0, cen[3] = {0.0, 0.0, 0.0};
    for (int64_t b = first[a]; b >= 0; b = link[b]) {
      ++size;
      ftot += flux[b];
      if (rad[b] > rmax) rmax = rad[b];
      for (int ax = 0; ax < 3; ++ax) {
        const double u = (double)(cells[3 * a + ax] +
                                  min_image((int64_t)cells[3 * b + ax] - cells[3 * a + ax], nn,
                                            periodic));
        cen[ax] += flux[b] * u;
      }
    }
    merged* o = &out[nout++];
    o->flux = ftot;
    o->radius = rmax;
    if (size == 1) {
      for (int ax = 0; ax < 3; ++ax) o->c[ax] = cells[3 * a + ax];
    } else {
      int64_t rnd[3];
      for (int ax = 0; ax < 3; ++ax) {
        const double cc = cen[ax] / ftot;
        const int64_t v = (int64_t)floor(cc + 0.5);
        rnd[ax] = periodic ? wrapi(v, nn) : v;
      }
      int64_t best = -1, bestd = 0;
      for (int64_t b = first[a]; b >= 0; b = link[b]) {
        int64_t d2 = 0;
        for (int ax = 0; ax < 3; ++ax) {
          const int64_t dd = min_image((int64_t)cells[3 * b + ax] - rnd[ax], nn, periodic);
          d2 += dd * dd;
        }
        if (best < 0 || d2 < bestd) {
          best = b;
          bestd = d2;
        }
      }
      for (int ax = 0; ax < 3; ++ax) o->c[ax] = cells[3 * best + ax];
    }
    o->key = ((int64_t)o->c[0] * nn + o->c[1]) * nn + o->c[2];
  }
  free(first);
  free(link);
  qsort(out, (size_t)nout, sizeof(merged), cmp_merged);
  for (int64_t q = 0; q < nout; ++q) {
    for (int ax = 0; ax < 3; ++ax) cells_out[3 * q + ax] = out[q].c[ax];
    flux_out[q] = out[q].flux;
    radius_out[q] = out[q].radius;
  }
  rc = nout;
done:
  free(cells);
  free(flux);
  free(rad);
  free(parent);
  free(out);
  return rc;
}
