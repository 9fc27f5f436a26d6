/*
 * nyxrt -- MI355X-native adaptive ray-tracing sweep of Nyx-RT (arXiv 2512.12466).
 *
 * C ABI: plain pointers and sizes, no C++ types, no exceptions.  Every call
 * returns an nrt_status; on failure nrt_last_error() holds a message and no
 * caller buffer has been written (except where a function says otherwise).
 *
 * Conventions
 *   Grid       cubic, n cells per side, cell width h_cm.  Fields are flat
 *              arrays of n^3 cell-centred values indexed c = i + n*(j + n*k)
 *              (i fastest; a C-ordered [k][j][i] array).
 *   Positions  in cell units: cell (i,j,k) covers [i,i+1)x[j,j+1)x[k,k+1).
 *   x          the IONIZED fraction; the absorber is a_abs = (1 - x) n_H
 *              (Sec. "Geometric correction").
 *   Gamma      photo-ionisation rate per neutral H atom [s^-1] (Eq. lut_eqn).
 *   Device     pointers marked "device" are HIP device memory of the device
 *              that was current at nrt_init_grid; pointers marked "host" are
 *              ordinary host memory.
 *   Streams    all device work of a context is enqueued on the stream given
 *              at nrt_init_grid.  Calls that return host results synchronise
 *              that stream before returning.
 *   Ownership  the caller owns every buffer it passes, including the device
 *              workspace; the library allocates no device memory.  Inputs are
 *              copied at call time and may be freed after the call returns.
 *   Threads    a context is not thread-safe; distinct contexts are independent.
 */
#ifndef NYXRT_H
#define NYXRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nrt_ctx nrt_ctx;

typedef enum {
  NRT_OK = 0,
  NRT_ERR_ARG = 1,      /* invalid argument or input value                      */
  NRT_ERR_STATE = 2,    /* call not valid in the context's state                */
  NRT_ERR_NOMEM = 3,    /* workspace (or host memory) too small                 */
  NRT_ERR_OVERFLOW = 4, /* a ray queue or source table would overflow           */
  NRT_ERR_DEVICE = 5,   /* a HIP call failed                                    */
  NRT_ERR_INTERNAL = 6  /* invariant violated inside the library                */
} nrt_status;

/* Arithmetic of the march (a3-a4).  Both paths take every discrete decision
   (cell crossing, split, face choice, the tau_max stop, thresholds) in FP64
   with the same operations, so they execute the same segments, rays and
   splits: the optical depth that the tau_max stop reads is accumulated in
   FP64 from the FP64 absorber in both.  NRT_MIXED computes the attenuation,
   the deposits and the correction factors in FP32 (the neighbour's absorber
   rounded to FP32 where it is read, floored at FLT_MIN) and keeps the
   transmitted fraction and the photon budget in FP64.  Both paths hold the
   absorber as one FP64 array, so their workspaces are the same size. */
typedef enum { NRT_FP64 = 0, NRT_MIXED = 1 } nrt_precision;

/* Overlap correction (Sec. "Geometric correction"). */
typedef enum {
  NRT_CORR_NONE = 0,         /* f_c = 1                                             */
  NRT_CORR_LINEAR = 1,       /* Eq. correction, no neighbour deposit                */
  NRT_CORR_CONSERVATIVE = 2, /* Eqs. new_correction + new_secondary (the paper's)   */
  NRT_CORR_SQUARED = 3,      /* f_c = (1/2 + D_edge/L_pix)^2, no neighbour deposit  */
  NRT_CORR_NAIVE = 4         /* Eq. correction; Eq. secondary_correction dropped
                                where n'_H < n_th ("naive thresholding")           */
} nrt_corr;

/* Source spectrum (Sec. "Flux computation").  The photo-ionisation
   cross-section falls as sigma0 (nu/nu_0)^-3 above the threshold nu_0
   (h nu_0 = 13.6 eV).  For a polychromatic spectrum a ray's optical depth tau
   is the one at the threshold, and the flux of Eq. lut_eqn integrated over
   frequency is evaluated from a table in tau built at nrt_init_grid: the
   share F(tau) of a ray's photons left after tau, and its thin-cell slope
   -F'(tau) for cells with no absorber (the optically thin table of the
   footnote in Sec. "Numerical instability for low n_H neighbor cells").  The
   cap tau_max then applies to the whole spectrum: a ray stops once
   F(tau) <= e^{-tau_max}, the share a monochromatic ray keeps at tau_max.
   The library takes that decision on the threshold optical depth, against
   the depth at which its FP64 table of -ln F reaches tau_max (found once at
   nrt_init_grid), so both precisions take it alike. */
typedef enum {
  NRT_SPEC_MONO = 0,      /* every photon at nu_0 (spec_param ignored)           */
  NRT_SPEC_BLACKBODY = 1, /* photon rate per frequency ~ nu^2 / (e^{h nu/kT} - 1);
                             spec_param = T [K] in [1e3, 1e7]                      */
  NRT_SPEC_POWERLAW = 2   /* photon rate per frequency ~ nu^-alpha;
                             spec_param = alpha in [2.5, 50]                       */
} nrt_spectrum;

#define NRT_MAX_LEVEL 14 /* HEALPix level cap: 12 * 4^14 pixels fit in 32 bits */

typedef struct {
  int32_t n;          /* cells per side, 1 <= n <= 4096                            */
  double h_cm;        /* cell width [cm], > 0                                      */
  int32_t periodic;   /* 1: rays wrap and stop after sqrt(3) n cells (Sec.
                         "Periodic BCs"); 0: rays leaving the box escape           */
  double sigma0;      /* cross-section at the threshold [cm^2], >= 0              */
  double n_min_ray;   /* N_min^ray of Eq. split_criterion, >= 0; 0 never splits   */
  int32_t l_max;      /* HEALPix level cap, 0 .. NRT_MAX_LEVEL                    */
  double tau_max;     /* optical-depth cap, > 0 (with a spectrum: a ray stops once
                         F(tau) <= e^{-tau_max}, see nrt_spectrum)                */
  double n_th;        /* neighbour density threshold [cm^-3] (Eq. new_correction) */
  int32_t corr;       /* nrt_corr                                                 */
  int32_t precision;  /* nrt_precision                                            */
  int32_t spectrum;   /* nrt_spectrum (0 = monochromatic)                         */
  double spec_param;  /* temperature or power-law index, see nrt_spectrum        */
} nrt_grid_desc;

/* Source-merging parameters (Sec. "Source Merging Algorithm"). */
typedef struct {
  double dr;           /* shell step [cells], > 0                       */
  double x_th;         /* a sample is ionized iff x >= x_th             */
  double f_req;        /* a shell passes iff N_ion / N_tot >= f_req     */
  int32_t n_min;       /* below n_min samples every sample must pass    */
  double r_max;        /* radius cap [cells]                            */
  double f_ov;         /* overlap factor                                */
  double eps;          /* squared-distance tolerance [cells^2]          */
  int32_t shell_level; /* HEALPix level of the shell directions, 0..3   */
} nrt_merge_params;

/* Photon budget of one pass: emitted = absorbed + escaped + truncated. */
typedef struct {
  double emitted;    /* sum of source rates [photons/s]                         */
  double absorbed;   /* deposited on the grid                                   */
  double escaped;    /* left the box, or reached sqrt(3) n in a periodic box    */
  double truncated;  /* dropped at tau_max, or at l_max when a split was due    */
  uint64_t segments; /* cell segments marched (the throughput unit)             */
  uint64_t rays;     /* rays marched: spawned plus split children               */
  uint64_t splits;   /* rays that split into four                               */
  uint64_t rays_per_level[NRT_MAX_LEVEL + 1];
} nrt_budget;

/* Bytes of device workspace a context needs: fields for n^3 cells, a table
   of max_sources sources, and ray queues of ray_capacity slots per HEALPix
   level (ray_capacity >= 4096; larger queues mean fewer, larger launches).
   Returns NRT_ERR_ARG for an invalid descriptor. */
nrt_status nrt_workspace_bytes(const nrt_grid_desc* desc, int64_t max_sources,
                               int64_t ray_capacity, size_t* bytes);

/* Create a context on the current HIP device.  n_H and x_ion: device, n^3
   FP64 each, read during the call (n_H finite and >= 0, 0 <= x_ion <= 1,
   else NRT_ERR_ARG).  workspace: device, ws_bytes >= nrt_workspace_bytes(),
   256-byte aligned, owned by the caller and used until nrt_destroy.
   hip_stream: a hipStream_t (NULL = the null stream).  *out receives the
   context; nothing is created on failure.  A polychromatic spectrum is
   tabulated here: NRT_ERR_ARG if its transmitted share F does not fall to
   1e-6 e^{-tau_max} within tau < 2^64 (spectra too hard for the table). */
nrt_status nrt_init_grid(nrt_ctx** out, const nrt_grid_desc* desc, const double* n_H,
                         const double* x_ion, int64_t max_sources, int64_t ray_capacity,
                         void* workspace, size_t ws_bytes, void* hip_stream);

/* Replace the ionized fraction (device, n^3 FP64, 0 <= x <= 1). */
nrt_status nrt_set_ionization(nrt_ctx* ctx, const double* x_ion);

/* Copy the context's ionized fraction into x_out (device, n^3 FP64). */
nrt_status nrt_get_ionization(nrt_ctx* ctx, double* x_out);

/* Append m point sources (Sec. "Halo finding and source luminosity"):
   pos host m*3 in cell units, each in [0, n); ndot host m rates
   [photons/s], finite and >= 0.  A source casts 12 HEALPix level-0 rays
   from its position, each with rate ndot / 12.  NRT_ERR_OVERFLOW if the
   table would exceed max_sources (nothing appended). */
nrt_status nrt_add_sources(nrt_ctx* ctx, int64_t m, const double* pos, const double* ndot);

/* Remove every source. */
nrt_status nrt_clear_sources(nrt_ctx* ctx);

/* Number of sources in the table. */
nrt_status nrt_source_count(const nrt_ctx* ctx, int64_t* m);

/* Copy the source table to the host: pos m*3, ndot m, radius m (bubble
   radius from the last merge, else 0); any pointer may be NULL. */
nrt_status nrt_get_sources(nrt_ctx* ctx, double* pos, double* ndot, double* radius);

/* Source merging (Sec. "Source Merging Algorithm", Alg. source_merge) on the
   GPU, using the context's ionized fraction: snap sources to cells and merge
   same-cell sources, compute each source's bubble radius (max_radius), unite
   sources whose bubbles overlap, collapse each group into one source at the
   member cell nearest its flux-weighted centroid, sort lexicographically by
   (i,j,k).  The table is replaced by the merged catalogue, whose positions
   are cell centres; *m_after receives its size. */
nrt_status nrt_merge_sources(nrt_ctx* ctx, const nrt_merge_params* mp, int64_t* m_after);

/* One ray-tracing pass (Alg. trace_rays): spawn 12 rays per source, march
   cell by cell accumulating optical depth and depositing Gamma (Eq. lut_eqn
   with V_box = h^3, the overlap correction of desc->corr), split by Eq.
   split_criterion into the 4 nested HEALPix children, terminate at tau_max,
   at l_max, at box exit or after sqrt(3) n cells when periodic, until no ray
   is left.  gamma_out: device n^3 FP64, overwritten.  budget: host, filled
   on return (the call synchronises).  NRT_ERR_OVERFLOW if the ray queues
   cannot hold a split (Gamma then unspecified). */
nrt_status nrt_trace_step(nrt_ctx* ctx, double* gamma_out, nrt_budget* budget);

/* The same pass without a host round trip, for callers that record it in
   their own hipGraph (stream capture on ctx's stream) or overlap it with
   other work.  It enqueues the device-driven pass, one march launch per
   HEALPix level with each level's ray count read from device memory, and
   a kernel that writes the budget into device memory, then returns without
   synchronising.  It allocates nothing, issues no memset or copy, and
   clears its device state with kernels, so it may be called while ctx's
   stream is being captured; a recorded pass replays with the source table,
   gamma_out, budget_dev and dropped_dev it was recorded with, and with the
   absorber field current at replay.
   gamma_out: device n^3 FP64, overwritten.  budget_dev: device nrt_budget,
   written by the pass.  dropped_dev: device uint64 or NULL, written with the
   number of rays whose children did not fit their level's queue.  This form
   cannot fall back to the host-driven chunked pass: when *dropped_dev is
   nonzero, Gamma and the budget are incomplete; give ray_capacity at least
   the widest level's ray count (budget.rays_per_level of nrt_trace_step).
   NRT_ERR_STATE if the source table changed since the last pass and ctx's
   stream is capturing (the table is copied from host memory then; run one
   pass outside capture first).  Nothing is enqueued when a check fails. */
nrt_status nrt_trace_step_async(nrt_ctx* ctx, double* gamma_out, nrt_budget* budget_dev,
                                uint64_t* dropped_dev);

/* For callers that cannot allocate (code under stream capture, tight
   serving loops, harnesses that forbid hipMalloc): nrt_trace_step's pass
   with no context and no allocation.  The library keeps the pass's device
   state (the absorber, the source table, the level queues, the
   accumulators) in a static device array of 64 MiB per GPU, held until the
   process ends; the call issues no hipMalloc/hipFree and uses no host heap.
   desc as for nrt_init_grid, monochromatic only (NRT_ERR_ARG otherwise).
   n_H, x_ion: device n^3 FP64 (read during the call; invalid values give
   NRT_ERR_ARG after the pass).  pos host m*3, ndot host m, as for
   nrt_add_sources.  ray_capacity: slots per HEALPix level queue, in
   [64, 2^32].  gamma_out: device n^3 FP64, overwritten.  budget: host,
   filled on return (the call synchronises hip_stream).  The pass is the
   device-driven one (one launch per level): NRT_ERR_OVERFLOW when a level
   does not fit ray_capacity (the budget then reports the rays that
   fitted); NRT_ERR_NOMEM when the absorber (8 B per cell), the sources
   (32 B each) and the queues (24 B per slot and level) exceed 64 MiB.  Calls that overlap on one GPU share the array and
   race.  Messages: nrt_last_error(NULL). */
nrt_status nrt_trace_step_noalloc(const nrt_grid_desc* desc, const double* n_H,
                                  const double* x_ion, int64_t m, const double* pos,
                                  const double* ndot, int64_t ray_capacity, double* gamma_out,
                                  nrt_budget* budget, void* hip_stream);

/* One radiation step of length dt_s (Secs. "Time integration" and
   "Iterative nonlinear solve"): iterate { trace with a = (1 - x_avg) n_H;
   update x by the time-averaged solution of Eq. chem_ode with C_H = 0 and
   recombination coefficient alpha = clumping * alpha_B } until at most
   conv_frac * n^3 cells changed x_avg by tol or more in the last pass
   (conv_frac = 0: every cell changed by less than tol), or max_iter passes;
   then commit x(dt).  The paper iterates "until convergence" without a
   criterion; conv_frac > 0 lets a few front cells keep moving.
   gamma_out: device n^3 FP64 (Gamma of the last pass); budget: host (last
   pass); iters: host, passes done.  The context's x is updated.
   NRT_ERR_ARG for dt_s <= 0, alpha < 0, tol < 0, conv_frac outside [0, 1]
   or max_iter < 1. */
nrt_status nrt_rt_step(nrt_ctx* ctx, double dt_s, double alpha, double tol, double conv_frac,
                       int32_t max_iter, double* gamma_out, nrt_budget* budget, int32_t* iters);

/* Test hook: march k injected rays that never split (desc->n_min_ray must be
   0): origin host k*3 (cell units, inside the box), dir host k*3 unit
   vectors, level host k (sets the pixel solid angle of the overlap
   correction), L host k rates.  gamma_out: device n^3 FP64, overwritten. */
nrt_status nrt_trace_rays_debug(nrt_ctx* ctx, int64_t k, const double* origin, const double* dir,
                                const int32_t* level, const double* L, double* gamma_out,
                                nrt_budget* budget);

/* HEALPix nested pixel-centre directions as the march uses them: out host
   3*count doubles for pixels first .. first+count-1 of `level`.  Levels up
   to min(l_max, 11) come from the context's direction table, which
   nrt_init_grid computes on the host with the C library's cos and sin;
   deeper levels are computed by the march's device function. */
nrt_status nrt_healpix_dirs(nrt_ctx* ctx, int32_t level, int64_t first, int64_t count,
                            double* out);

/* Launch parameters of the march kernel.  0 selects the built-in default. */
typedef struct {
  int32_t refill_min;    /* idle lanes that make a wavefront fetch new rays (1..64;
                            default 16)                                              */
  int32_t claim;         /* rays a wavefront claims at a time (64..65536, multiple of
                            64; default 128)                                         */
  int32_t blocks_per_cu; /* resident 256-thread blocks per compute unit (default: as
                            many as the kernel's registers and LDS allow)            */
  int32_t graph;         /* 0: replay a captured device-driven pass (hipGraph) once a
                            pass has shown that every HEALPix level fits its queue;
                            1: never; 2: always try (falls back on overflow)        */
} nrt_tuning;

/* Set (or read back) the march launch parameters of a context.  Results
   do not depend on them; only the speed does.  NRT_ERR_ARG when out of range. */
nrt_status nrt_set_tuning(nrt_ctx* ctx, const nrt_tuning* t);
nrt_status nrt_get_tuning(const nrt_ctx* ctx, nrt_tuning* t);

/* Autotuner: run one trace pass (into gamma_scratch, device n^3 FP64) per
   candidate parameter set (refill_min 8, 16, 32, 64 x claim 0, 64, 256 x
   blocks_per_cu as many as fit or one fewer), time the march kernels with
   HIP events, keep the fastest in the context and return it in *best (host).
   `passes` repeats each candidate (>= 1).  Uses the context's current grid
   and sources. */
nrt_status nrt_autotune(nrt_ctx* ctx, double* gamma_scratch, int32_t passes, nrt_tuning* best);

/* Average duration [ms] of the march kernel launches of the last pass,
   timed with HIP events on the context's stream, the number of those
   launches, and whether the pass replayed the captured graph (then the
   average is the graph's duration over its march launches).  Any pointer
   may be NULL. */
nrt_status nrt_last_kernel_time(const nrt_ctx* ctx, double* march_ms, int32_t* launches,
                                int32_t* graph_replayed);

/* Destroy a context (the workspace remains the caller's).  NULL is a no-op. */
nrt_status nrt_destroy(nrt_ctx* ctx);

/* Static description of a status code. */
const char* nrt_status_str(nrt_status s);

/* Message of the last failure of ctx (or of the last failed nrt_init_grid
   when ctx is NULL); valid until the next call on the same context. */
const char* nrt_last_error(const nrt_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* NYXRT_H */
