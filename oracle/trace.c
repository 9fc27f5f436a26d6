/*
 * Oracle (test infrastructure only): one adaptive ray-tracing pass in FP64.
 *
 * Follows the paper in this order:
 *   spawn      12 HEALPix level-0 rays per source (Sec. "Adaptive ray
 *              tracing", Alg. trace_rays spawn_rays, Fig. raysplit (a)),
 *              each carrying L = Ndot / 12 (reading: the paper divides L
 *              evenly at splits and is silent about the spawn).
 *   raymarch   Alg. functors: march cell by cell with the Amanatides-Woo
 *              traversal while the ray does not need to split, is inside the
 *              domain and has travelled less than sqrt(3) L_box.
 *   flux       Eq. lut_eqn with V_shell replaced by V_box = h^3 (footnote
 *              to Alg. functors).  Monochromatic at threshold:
 *              Gamma = L e^{-tau} (1 - e^{-dtau}) / (n_HI h^3), and its
 *              n_HI -> 0 limit L e^{-tau} sigma0 dl / h^3 (footnote in
 *              Sec. "Numerical instability for low n_H neighbor cells").
 *              With a spectrum (spectrum.c), tau is the threshold optical
 *              depth and Gamma = L D(tau, dtau) / (n_HI h^3), with the limit
 *              L G(tau) sigma0 dl / h^3; a ray carries L F(tau) photons.
 *   depth      Eq. optical_depth with the absorber a_abs = (1 - x) n_H of
 *              Sec. "Geometric correction" (reading: the printed integrand
 *              "sigma x n_HI" is garbled; a_abs is used).
 *   correction Eqs. correction, secondary_correction, new_correction and
 *              new_secondary (the paper's final "conservative
 *              thresholding" is ORC_CORR_CONSERVATIVE).
 *   ray_fltr   terminate on tau >= tau_max, on level l_max needing a split,
 *              and on s >= sqrt(3) L_box in the periodic case.  With a
 *              spectrum the optical-depth cap applies to the whole spectrum:
 *              the ray stops once the share of its photons left, F(tau),
 *              is at most e^{-tau_max}, the share a monochromatic ray keeps
 *              at tau_max (reading: the paper caps the optical depth of a
 *              monochromatic ray; at the threshold a hard spectrum would
 *              still carry a sizeable share of its photons there).
 *   s_copy /   4 children at level l+1, pixel 4 pix + k, same s and tau,
 *   s_tsfm     L / 4, restarting at o + s d_child (Alg. functors).
 *
 * Readings where the paper is silent:
 *   - The split test Omega_c / Omega(l) < N_min with Omega_c = 1/s^2 (cell
 *     units, s = distance from the source) is evaluated as s*s > r2[l],
 *     r2[l] = 1 / (N_min * Omega(l)), at every cell boundary before the ray
 *     advances (so a child may split again at once).  Equality does not
 *     split.
 *   - Stop tests run in the order: s >= s_max, tau >= tau_max, split.
 *   - tau_max is tested at every boundary, not only after the march.
 *   - A ray at l_max that needs to split is terminated (its photons are
 *     booked as truncated).
 *   - Non-periodic boxes: a ray leaving [0,n)^3 escapes; a neighbour cell
 *     outside the box is not a valid neighbour.
 *   - D_edge is the smallest perpendicular distance from the segment
 *     midpoint to the six faces of the current cell; the neighbour c' lies
 *     across that face.  Ties: lowest axis; on one axis, the face on the
 *     side the ray travels (+ when the component is zero).
 *   - L_pix = r_m sqrt(Omega(l)), r_m the midpoint's distance from the source.
 *   - A neighbour is usable iff it is in the domain, n'_H >= n_th and
 *     a'_abs > 0 (a fully ionized neighbour would divide by zero).
 *   - Start cell of a ray at q = o + s d: floor(q) per axis, except that an
 *     exact integer with a negative component belongs to the cell below.
 *   - Segment length ds = max(0, t_next - s); a zero-length segment still
 *     counts as a segment and deposits nothing.
 *
 * Every comparison that decides a cell, a face or a split uses only
 * correctly rounded +, -, *, / and sqrt (the file is compiled with
 * -ffp-contract=off), so any other FP64 implementation of the same formulas
 * takes the same decisions.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"
#include "spectrum.h"

typedef struct {
  int level;
  uint64_t pix;
  double s, tau, L;
} orc_ray;

typedef struct {
  orc_ray* data;
  int64_t size, cap;
} orc_stack;

static int stack_push(orc_stack* st, orc_ray r) {
  if (st->size == st->cap) {
    int64_t cap = st->cap ? 2 * st->cap : 1024;
    orc_ray* d = (orc_ray*)realloc(st->data, (size_t)cap * sizeof(orc_ray));
    if (!d) return -1;
    st->data = d;
    st->cap = cap;
  }
  st->data[st->size++] = r;
  return 0;
}

typedef struct {
  const orc_params* p;
  const double* n_H;
  const double* a; /* absorber (1 - x) n_H */
  orc_spectrum spec;
  double t_min; /* e^{-tau_max} */
  double s_max;
  double h3;
  double r2split[ORC_MAX_LEVEL + 1];
  double sqrt_omega[ORC_MAX_LEVEL + 1];
} orc_grid;

typedef struct {
  int64_t max_log, n_log;
  int64_t* cell;
  double* ds;
  int64_t* ijk;
} orc_log;

static int64_t wrap_index(int64_t i, int64_t n) { return ((i % n) + n) % n; }

static int inside(const int64_t i[3], int64_t n) {
  return i[0] >= 0 && i[0] < n && i[1] >= 0 && i[1] < n && i[2] >= 0 && i[2] < n;
}

static int64_t flat_index(const int64_t i[3], int64_t n) {
  return wrap_index(i[0], n) + n * (wrap_index(i[1], n) + n * wrap_index(i[2], n));
}

/* parametric distance from the source to the next plane of axis a */
static double plane_t(double o, double d, int64_t i) {
  if (d > 0.0) return ((double)(i + 1) - o) / d;
  if (d < 0.0) return ((double)i - o) / d;
  return INFINITY;
}

/* photons per unit L left after threshold optical depth tau */
static double transmitted(const orc_grid* g, double tau) {
  return g->p->spectrum == ORC_SPEC_MONO ? exp(-tau) : orc_spectrum_F(&g->spec, tau);
}

static int grid_setup(orc_grid* g, const orc_params* p, const double* n_H, const double* a) {
  if (orc_spectrum_init(&g->spec, p->spectrum, p->spec_param)) return 1;
  g->p = p;
  g->n_H = n_H;
  g->a = a;
  g->s_max = p->periodic ? sqrt(3.0) * (double)p->n : INFINITY;
  g->t_min = exp(-p->tau_max);
  g->h3 = p->h_cm * p->h_cm * p->h_cm;
  for (int l = 0; l <= ORC_MAX_LEVEL; ++l) {
    /* Omega(l) = 4 pi / (12 * 4^l), Eq. split_criterion */
    const double omega = (4.0 * M_PI) / (12.0 * ldexp(1.0, 2 * l));
    g->sqrt_omega[l] = sqrt(omega);
    g->r2split[l] = p->n_min_ray > 0.0 ? 1.0 / (p->n_min_ray * omega) : INFINITY;
  }
  return 0;
}

/* One cell segment [s, t_next] of a ray in unwrapped cell i: Eq. lut_eqn,
   Eq. optical_depth and the overlap correction.  Returns the segment's
   optical depth. */
static double segment(const orc_grid* g, const double o[3], const double d[3], int level,
                      const int64_t i[3], double s, double t_next, double ds, double tau,
                      double L, double* gamma, orc_budget* b) {
  const orc_params* p = g->p;
  const int64_t n = p->n;
  const int64_t c = flat_index(i, n);
  const double a_c = g->a[c];
  const double dl = ds * p->h_cm;               /* path length in cm       */
  const double dtau = p->sigma0 * a_c * dl;      /* Eq. optical_depth       */
  double G;                                      /* Eq. lut_eqn, V = h^3    */
  double dN;                                     /* photons/s absorbed      */
  if (p->spectrum == ORC_SPEC_MONO) {
    const double P = L * exp(-tau);              /* photons/s entering      */
    dN = P * (-expm1(-dtau));
    if (a_c > 0.0)
      G = dN / (a_c * g->h3);
    else
      G = P * p->sigma0 * dl / g->h3;
  } else {
    dN = L * orc_spectrum_D(&g->spec, tau, dtau);
    if (a_c > 0.0)
      G = dN / (a_c * g->h3);
    else
      G = L * orc_spectrum_G(&g->spec, tau) * p->sigma0 * dl / g->h3;
  }
  b->absorbed += dN;

  double fc = 1.0;
  int secondary = 0;
  int64_t c2 = -1;
  double a2 = 0.0;
  if (p->corr != ORC_CORR_NONE) {
    const double rm = 0.5 * (s + t_next); /* midpoint distance */
    double m[3];
    for (int ax = 0; ax < 3; ++ax) m[ax] = o[ax] + rm * d[ax];
    const double lpix = rm * g->sqrt_omega[level];
    double dedge = INFINITY;
    int fax = 0, fdir = 1;
    for (int ax = 0; ax < 3; ++ax) {
      const double dm = m[ax] - (double)i[ax];
      const double dp = (double)(i[ax] + 1) - m[ax];
      double da;
      int sa;
      if (dm < dp) {
        da = dm;
        sa = -1;
      } else if (dp < dm) {
        da = dp;
        sa = 1;
      } else {
        da = dp;
        sa = d[ax] < 0.0 ? -1 : 1;
      }
      if (da < dedge) {
        dedge = da;
        fax = ax;
        fdir = sa;
      }
    }
    int64_t j[3] = {i[0], i[1], i[2]};
    j[fax] += fdir;
    const int in_domain = p->periodic || inside(j, n);
    int usable = 0;
    if (in_domain) {
      c2 = flat_index(j, n);
      a2 = g->a[c2];
      usable = g->n_H[c2] >= p->n_th && a2 > 0.0;
    }
    const int near = dedge < 0.5 * lpix;
    switch (p->corr) {
      case ORC_CORR_LINEAR:
        if (near) fc = 0.5 + dedge / lpix;
        break;
      case ORC_CORR_CONSERVATIVE:
        if (near && usable) fc = 0.5 + dedge / lpix;
        secondary = usable;
        break;
      case ORC_CORR_SQUARED:
        if (near) {
          const double f = 0.5 + dedge / lpix;
          fc = f * f;
        }
        break;
      case ORC_CORR_NAIVE:
        if (near) fc = 0.5 + dedge / lpix;
        secondary = usable;
        break;
      default:
        break;
    }
  }
  gamma[c] += fc * G;
  if (secondary) {
    const double f2 = (1.0 - fc) * (a_c / a2); /* Eq. new_secondary */
    gamma[c2] += f2 * G;
  }
  return dtau;
}

/* raymarch of Alg. functors for one ray, followed by ray_fltr and the split
   (children pushed on st).  can_split = 0 for injected rays. */
static int march(const orc_grid* g, const double o[3], const double d[3], orc_ray r,
                 int can_split, double* gamma, orc_budget* b, orc_stack* st, orc_log* lg) {
  const orc_params* p = g->p;
  const int64_t n = p->n;
  int64_t i[3];
  double t[3];
  int step[3];
  for (int ax = 0; ax < 3; ++ax) {
    const double q = o[ax] + r.s * d[ax];
    const double f = floor(q);
    i[ax] = (int64_t)f;
    if (q == f && d[ax] < 0.0) i[ax] -= 1;
    step[ax] = d[ax] > 0.0 ? 1 : (d[ax] < 0.0 ? -1 : 0);
    t[ax] = plane_t(o[ax], d[ax], i[ax]);
  }
  double s = r.s, tau = r.tau;
  if (!p->periodic && !inside(i, n)) {
    b->escaped += r.L * transmitted(g, tau);
    return 0;
  }
  for (;;) {
    if (p->periodic && s >= g->s_max) {
      b->escaped += r.L * transmitted(g, tau);
      return 0;
    }
    if (p->spectrum == ORC_SPEC_MONO ? tau >= p->tau_max : transmitted(g, tau) <= g->t_min) {
      b->truncated += r.L * transmitted(g, tau);
      return 0;
    }
    if (can_split && s * s > g->r2split[r.level]) {
      if (r.level >= p->l_max) {
        b->truncated += r.L * transmitted(g, tau);
        return 0;
      }
      b->splits += 1;
      for (int k = 0; k < 4; ++k) {
        orc_ray ch = {r.level + 1, 4 * r.pix + (uint64_t)k, s, tau, r.L / 4.0};
        if (stack_push(st, ch)) return -1;
      }
      return 0;
    }
    int ax = 0;
    if (t[1] < t[ax]) ax = 1;
    if (t[2] < t[ax]) ax = 2;
    const double t_next = t[ax];
    double ds = t_next - s;
    if (ds < 0.0) ds = 0.0;
    if (lg && lg->cell && lg->n_log < lg->max_log) {
      lg->cell[lg->n_log] = flat_index(i, n);
      lg->ds[lg->n_log] = ds;
      if (lg->ijk)
        for (int q = 0; q < 3; ++q) lg->ijk[3 * lg->n_log + q] = i[q];
    }
    if (lg) lg->n_log += 1;
    const double dtau = segment(g, o, d, r.level, i, s, t_next, ds, tau, r.L, gamma, b);
    tau += dtau;
    s = t_next;
    i[ax] += step[ax];
    t[ax] = plane_t(o[ax], d[ax], i[ax]);
    b->segments += 1;
    if (!p->periodic && !inside(i, n)) {
      b->escaped += r.L * transmitted(g, tau);
      return 0;
    }
  }
}

static int check_params(const orc_params* p) {
  if (!p || p->n < 1 || !(p->h_cm > 0.0) || !(p->sigma0 >= 0.0)) return 1;
  if (p->l_max < 0 || p->l_max >= ORC_MAX_LEVEL) return 1;
  if (!(p->tau_max > 0.0) || !(p->n_min_ray >= 0.0)) return 1;
  if (p->corr < ORC_CORR_NONE || p->corr > ORC_CORR_NAIVE) return 1;
  if (p->spectrum < ORC_SPEC_MONO || p->spectrum > ORC_SPEC_POWERLAW) return 1;
  return 0;
}

static double* make_absorber(int64_t ncell, const double* n_H, const double* x) {
  double* a = (double*)malloc((size_t)ncell * sizeof(double));
  if (!a) return NULL;
  for (int64_t c = 0; c < ncell; ++c) a[c] = (1.0 - x[c]) * n_H[c];
  return a;
}

/* ---- multi-threaded pass over sources ---- */
typedef struct {
  const orc_grid* g;
  int64_t m;
  const double* pos;
  const double* ndot;
  int64_t* next; /* shared source counter */
  pthread_mutex_t* lock;
  double* gamma;  /* private */
  orc_budget b;   /* private */
  int err;
} orc_worker;

static void* worker_main(void* arg) {
  orc_worker* w = (orc_worker*)arg;
  orc_stack st = {NULL, 0, 0};
  for (;;) {
    pthread_mutex_lock(w->lock);
    const int64_t k = (*w->next)++;
    pthread_mutex_unlock(w->lock);
    if (k >= w->m) break;
    const double* o = w->pos + 3 * k;
    for (int pix = 0; pix < 12; ++pix) {
      orc_ray r = {0, (uint64_t)pix, 0.0, 0.0, w->ndot[k] / 12.0};
      if (stack_push(&st, r)) { w->err = 1; goto done; }
    }
    while (st.size > 0) {
      orc_ray r = st.data[--st.size];
      double d[3];
      orc_pix2vec_nest(r.level, r.pix, d);
      w->b.rays += 1;
      w->b.rays_per_level[r.level] += 1;
      if (march(w->g, o, d, r, 1, w->gamma, &w->b, &st, NULL)) { w->err = 1; goto done; }
    }
  }
done:
  free(st.data);
  return NULL;
}

static void budget_add(orc_budget* to, const orc_budget* from) {
  to->absorbed += from->absorbed;
  to->escaped += from->escaped;
  to->truncated += from->truncated;
  to->segments += from->segments;
  to->rays += from->rays;
  to->splits += from->splits;
  for (int l = 0; l <= ORC_MAX_LEVEL; ++l) to->rays_per_level[l] += from->rays_per_level[l];
}

int orc_trace(const orc_params* p, const double* n_H, const double* x, int64_t m,
              const double* pos, const double* ndot, int nthreads, double* gamma,
              orc_budget* b) {
  if (check_params(p) || m < 0 || !n_H || !x || !gamma || !b) return 1;
  const int64_t n = p->n, ncell = n * n * n;
  for (int64_t k = 0; k < m; ++k) {
    for (int ax = 0; ax < 3; ++ax) {
      const double q = pos[3 * k + ax];
      if (!(q >= 0.0 && q < (double)n)) return 1;
    }
    if (!(ndot[k] >= 0.0) || !isfinite(ndot[k])) return 1;
  }
  memset(b, 0, sizeof(*b));
  for (int64_t k = 0; k < m; ++k) b->emitted += ndot[k];
  memset(gamma, 0, (size_t)ncell * sizeof(double));
  if (m == 0) return 0;

  double* a = make_absorber(ncell, n_H, x);
  if (!a) return 2;
  orc_grid g;
  if (grid_setup(&g, p, n_H, a)) {
    free(a);
    return 1;
  }

  /* private FP64 Gamma per thread, capped at ~16 GB in total */
  int64_t nt = nthreads < 1 ? 1 : nthreads;
  const int64_t cap = (int64_t)(16e9 / (8.0 * (double)ncell));
  if (nt > cap) nt = cap < 1 ? 1 : cap;
  if (nt > m) nt = m;
  orc_worker* w = (orc_worker*)calloc((size_t)nt, sizeof(orc_worker));
  pthread_t* th = (pthread_t*)calloc((size_t)nt, sizeof(pthread_t));
  pthread_mutex_t lock;
  pthread_mutex_init(&lock, NULL);
  int64_t next = 0;
  int err = (!w || !th);
  for (int64_t q = 0; q < nt && !err; ++q) {
    w[q].g = &g;
    w[q].m = m;
    w[q].pos = pos;
    w[q].ndot = ndot;
    w[q].next = &next;
    w[q].lock = &lock;
    w[q].gamma = (double*)calloc((size_t)ncell, sizeof(double));
    if (!w[q].gamma) err = 1;
  }
  if (!err) {
    for (int64_t q = 0; q < nt; ++q) pthread_create(&th[q], NULL, worker_main, &w[q]);
    for (int64_t q = 0; q < nt; ++q) pthread_join(th[q], NULL);
    /* reduction in a fixed thread order */
    for (int64_t q = 0; q < nt; ++q) {
      if (w[q].err) err = 1;
      for (int64_t c = 0; c < ncell; ++c) gamma[c] += w[q].gamma[c];
      budget_add(b, &w[q].b);
    }
  }
  for (int64_t q = 0; w && q < nt; ++q) free(w[q].gamma);
  free(w);
  free(th);
  free(a);
  orc_spectrum_free(&g.spec);
  pthread_mutex_destroy(&lock);
  return err ? 2 : 0;
}

int orc_trace_rays(const orc_params* p, const double* n_H, const double* x, int64_t k,
                   const double* origin, const double* dir, const int32_t* level,
                   const double* L, double* gamma, orc_budget* b, int64_t max_log,
                   int64_t* log_cell, double* log_ds, int64_t* log_ijk, int64_t* n_log) {
  if (check_params(p) || p->n_min_ray != 0.0 || k < 0 || !gamma || !b) return 1;
  const int64_t n = p->n, ncell = n * n * n;
  for (int64_t r = 0; r < k; ++r)
    if (level[r] < 0 || level[r] > ORC_MAX_LEVEL || !(L[r] >= 0.0)) return 1;
  memset(b, 0, sizeof(*b));
  memset(gamma, 0, (size_t)ncell * sizeof(double));
  double* a = make_absorber(ncell, n_H, x);
  if (!a) return 2;
  orc_grid g;
  if (grid_setup(&g, p, n_H, a)) {
    free(a);
    return 1;
  }
  orc_log lg = {max_log, 0, log_cell, log_ds, log_ijk};
  for (int64_t r = 0; r < k; ++r) {
    b->emitted += L[r];
    orc_ray ray = {level[r], 0, 0.0, 0.0, L[r]};
    b->rays += 1;
    b->rays_per_level[level[r]] += 1;
    march(&g, origin + 3 * r, dir + 3 * r, ray, 0, gamma, b, NULL, &lg);
  }
  if (n_log) *n_log = lg.n_log;
  free(a);
  orc_spectrum_free(&g.spec);
  return 0;
}
