/*
 * Oracle for the Nyx-RT adaptive ray-tracing sweep (arXiv 2512.12466).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, serial-per-ray FP64 CPU
 * implementation written directly from the paper.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  The
 * GPU library shares no source, header, table or helper with it, and neither
 * includes nor links the other.
 *
 * Units: positions and lengths are in cell units (cell (i,j,k) covers
 * [i,i+1)x[j,j+1)x[k,k+1)); h_cm converts to cm.  Fields are cell-centred,
 * flat arrays indexed c = i + n*(j + n*k).  x is the IONIZED fraction
 * (Sec. "Geometric correction": a_abs = (1-x) n_H).
 *
 * What each function follows:
 *   orc_pix2vec_nest  HEALPix nested pixel centres (Gorski et al. 2005, the
 *                     pixelisation cited in Sec. "Adaptive ray tracing").
 *   orc_trace         Alg. trace_rays with the functors of Alg. functors,
 *                     flux from Eq. lut_eqn (V_box = h^3; monochromatic, or
 *                     integrated over a photon spectrum in spectrum.c),
 *                     optical depth from Eq. optical_depth with a_abs, split
 *                     test Eq. split_criterion, overlap correction
 *                     Eqs. correction / secondary_correction / new_correction /
 *                     new_secondary, periodic rule of Sec. "Periodic BCs".
 *   orc_trace_rays    the same march for injected rays with no splitting.
 *   orc_dedupe_sort, orc_max_radius, orc_merge_sources
 *                     Sec. "Source Merging Algorithm" and Alg. source_merge.
 *   orc_spectrum_eval the frequency integrals of Eq. lut_eqn against the
 *                     threshold optical depth (Sec. "Flux computation").
 *   orc_chem_update, orc_rt_step
 *                     Eq. chem_ode with the time-averaged integration of
 *                     C2-Ray (Sec. "Time integration") and the fixed-point
 *                     iteration of Sec. "Iterative nonlinear solve".
 *
 * The readings taken where the paper is silent or garbled are listed in
 * the comments of the functions that take them.
 */
#ifndef NYXRT_ORACLE_H
#define NYXRT_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* overlap-correction variants (Sec. "Geometric correction") */
enum {
  ORC_CORR_NONE = 0,         /* no correction: f_c = 1                          */
  ORC_CORR_LINEAR = 1,       /* Eq. correction only, nothing into the neighbour */
  ORC_CORR_CONSERVATIVE = 2, /* Eqs. new_correction + new_secondary (default)   */
  ORC_CORR_SQUARED = 3,      /* f_c squared (Wise & Abel), no neighbour deposit */
  ORC_CORR_NAIVE = 4         /* Eq. correction always; Eq. secondary_correction
                                dropped when n'_H < n_th ("naive thresholding")  */
};

/* source spectra (Sec. "Flux computation"); the cross-section is
   sigma_nu = sigma0 (nu / nu_0)^-3 */
enum {
  ORC_SPEC_MONO = 0,      /* all photons at the threshold nu_0                 */
  ORC_SPEC_BLACKBODY = 1, /* photon spectrum ~ nu^2 / (e^{h nu / k T} - 1),
                             param = T [K] in [1e3, 1e7], h nu_0 = 13.6 eV     */
  ORC_SPEC_POWERLAW = 2   /* photon spectrum ~ nu^-alpha, param = alpha in
                             [2.5, 50]                                         */
};

typedef struct {
  int32_t n;          /* cells per side                                   */
  double h_cm;        /* cell width in cm                                 */
  int32_t periodic;   /* 1: rays wrap and stop at sqrt(3) n; 0: escape    */
  double sigma0;      /* photo-ionisation cross-section at threshold, cm^2 */
  double n_min_ray;   /* N_min^ray of Eq. split_criterion; 0 = never split */
  int32_t l_max;      /* HEALPix level cap                                */
  double tau_max;     /* optical-depth cap; with a spectrum the ray stops
                         once F(tau) <= e^{-tau_max}                      */
  double n_th;        /* neighbour density threshold, cm^-3               */
  int32_t corr;       /* ORC_CORR_*                                       */
  int32_t spectrum;   /* ORC_SPEC_*; a ray's tau is at the threshold      */
  double spec_param;  /* temperature or power-law index (see ORC_SPEC_*)  */
} orc_params;

#define ORC_MAX_LEVEL 24

typedef struct {
  double emitted;    /* sum of source rates                     */
  double absorbed;   /* photons/s deposited on the grid         */
  double escaped;    /* photons/s leaving (box exit or s_max)   */
  double truncated;  /* photons/s dropped at tau_max or l_max   */
  uint64_t segments; /* executed cell segments                  */
  uint64_t rays;     /* rays marched (spawned + split children) */
  uint64_t splits;   /* parent rays that split                  */
  uint64_t rays_per_level[ORC_MAX_LEVEL + 1];
} orc_budget;

/* HEALPix nested-scheme pixel centre of pixel `pix` at level `level`
   (N_side = 2^level) as a unit vector. */
void orc_pix2vec_nest(int level, uint64_t pix, double v[3]);

/* One trace pass.  n_H, x: n^3 FP64.  pos: m*3 cell units in [0,n); ndot:
   m rates (photons/s).  gamma: n^3 output, overwritten.  nthreads >= 1.
   Returns 0 on success, nonzero on bad arguments or allocation failure. */
int orc_trace(const orc_params* p, const double* n_H, const double* x,
              int64_t m, const double* pos, const double* ndot,
              int nthreads, double* gamma, orc_budget* b);

/* Injected rays, never split (for geometry and attenuation pins): ray r
   starts at origin[3r] (s = 0) along the unit vector dir[3r] with rate L[r];
   level[r] sets the pixel solid angle used by the overlap correction.
   If log_cell is non-NULL, up to max_log segments are logged in order
   (wrapped flat cell index, segment length ds in cells, unwrapped cell ijk
   into log_ijk[3*]) and *n_log receives the number of segments. */
int orc_trace_rays(const orc_params* p, const double* n_H, const double* x,
                   int64_t k, const double* origin, const double* dir,
                   const int32_t* level, const double* L,
                   double* gamma, orc_budget* b,
                   int64_t max_log, int64_t* log_cell, double* log_ds,
                   int64_t* log_ijk, int64_t* n_log);

/* Frequency integrals of Eq. lut_eqn per unit photon rate, at threshold
   optical depths tau[i] (and cell depths dtau[i], may be NULL = 0):
   F = photons left, D = photons a cell absorbs, G = the thin-cell limit
   D / dtau as dtau -> 0.  Any output may be NULL.  Returns nonzero on a bad
   spectrum. */
int orc_spectrum_eval(int32_t kind, double param, int64_t k, const double* tau,
                      const double* dtau, double* F, double* D, double* G);

/* ---------------- source merging ---------------- */
typedef struct {
  double dr;        /* shell step (cells)                             */
  double x_th;      /* ionized-sample threshold                       */
  double f_req;     /* required ionized share of a shell              */
  int32_t n_min;    /* below this many samples every one must pass    */
  double r_max;     /* hard cap on the bubble radius (cells)          */
  double f_ov;      /* overlap factor                                 */
  double eps;       /* squared-distance tolerance (cells^2)           */
  int32_t shell_level; /* HEALPix level of the shell sample directions */
} orc_merge_params;

/* Snap m sources to cells (floor of position), merge sources that share a
   cell by summing rates, sort lexicographically by (i,j,k).  cells_out:
   m*3, flux_out: m.  Returns the deduplicated count (< 0 on error). */
int64_t orc_dedupe_sort(int32_t n, int64_t m, const double* pos,
                        const double* ndot, int32_t* cells_out,
                        double* flux_out);

/* Bubble radius of each (cell-snapped) source, Alg. source_merge max_radius. */
int orc_max_radius(const orc_merge_params* mp, int32_t n, int32_t periodic,
                   const double* x, int64_t m, const int32_t* cells,
                   double* radius_out);

/* Full merge: dedupe+sort, max_radius, union-find, collapse, sort.
   Outputs at most m entries; returns the merged count (< 0 on error). */
int64_t orc_merge_sources(const orc_merge_params* mp, int32_t n,
                          int32_t periodic, const double* x, int64_t m,
                          const double* pos, const double* ndot,
                          int32_t* cells_out, double* flux_out,
                          double* radius_out);

/* ---------------- chemistry ---------------- */
/* Per-cell time-averaged update of Eq. chem_ode over dt for fixed Gamma
   (C_H = 0): x0 -> x_new (end of step) and x_avg (step average).
   n_e = x_avg * n_H is iterated per cell.  alpha = clumping * alpha_B. */
void orc_chem_update(int64_t ncell, const double* gamma, const double* n_H,
                     const double* x0, double dt, double alpha,
                     const double* x_avg_guess, double* x_new, double* x_avg);

/* One radiation step: iterate { trace with a = (1 - x_avg) n_H ; chemistry }
   until at most conv_frac * n^3 cells changed x_avg by tol or more in the
   last iteration (conv_frac = 0: every cell changed by less than tol), or
   max_iter iterations; commit x <- x(dt).
   x: in/out n^3.  gamma: out (last trace).  iters: out.  Returns 0 on success. */
int orc_rt_step(const orc_params* p, const double* n_H, double* x,
                int64_t m, const double* pos, const double* ndot,
                double dt, double alpha, double tol, double conv_frac, int max_iter,
                int nthreads, double* gamma, orc_budget* b, int* iters);

#ifdef __cplusplus
}
#endif
#endif
