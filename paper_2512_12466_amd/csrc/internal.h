// Internal declarations of the nyxrt library: context, workspace layout,
// kernel argument blocks and kernel launchers.  Host code only sees the
// launchers; every kernel lives in the .hip file that launches it.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "nyxrt.h"

namespace nrt {

constexpr int kMaxLevel = NRT_MAX_LEVEL;
constexpr int kBlock = 256;  // threads per block of the march kernels (4 waves)

// One ray in a level queue (structure of arrays, 24 bytes per ray).  The
// HEALPix level is the queue's, the rate follows from the source and level,
// and the direction from (level, pix).  w is the optical depth tau at the
// ionization threshold, accumulated in FP64 in both precisions (it carries
// the tau_max decision).
struct RayQueue {
  uint32_t* src;
  uint32_t* pix;
  double* s;
  double* w;
};

// Polychromatic sources (Sec. "Flux computation"): Phi(tau) = -ln F(tau),
// F the share of a ray's photons left after threshold optical depth tau, is
// tabulated on the octaves [2^e, 2^(e+1)) of 1 + tau, each cut into
// kSpecSub equal intervals, for e < kSpecMaxOctaves.  Interval q = e kSpecSub
// + m covers 1 + tau in 2^e [1 + m/kSpecSub, 1 + (m+1)/kSpecSub); its local
// coordinate x in [0, 1) and index follow from the bits of 1 + tau, and
// Phi = c0 + c1 x + ... + c5 x^5 there (quintic Hermite through Phi, Phi'
// and Phi'' at both ends).
constexpr int kSpecLog2Sub = 6;
constexpr int kSpecSub = 1 << kSpecLog2Sub;
constexpr int kSpecMaxOctaves = 64;
constexpr int kSpecNodes = kSpecMaxOctaves * kSpecSub + 1;

// FP64 record of an interval: c1..c5, c0, padding (64 B)
struct SpecRec64 {
  double c[8];
};
// mixed-path record: c1..c5 in FP32, c0 in FP64 (32 B)
struct SpecRec32 {
  float c[6];
  double c0;
};

// Device accumulators of one pass.
struct Accum {
  double absorbed, escaped, truncated, pad;
  unsigned long long segments;
  unsigned long long overflow;
  unsigned long long invalid;  // input cells failing validation
  unsigned long long claim;  // rays claimed so far in the current march launch
  unsigned long long out_count[kMaxLevel + 2];  // rays pushed into each level queue
  unsigned long long chem_changed;  // cells whose x_avg moved by the tolerance or more
  unsigned long long claim_lv[kMaxLevel + 2];  // claim counters of a device-driven pass
};

// State of a radiation step's Gamma <-> x iteration when its passes replay
// a captured graph: written by k_rt_check at the end of every pass, read by
// the host once per batch of replays.  Once `done` is set, every kernel of a
// later replay returns at once.
struct RtState {
  unsigned long long done;      // 1 once the iteration has stopped
  unsigned long long iters;     // passes done
  unsigned long long changed;   // cells whose x_avg moved by tol or more (last pass)
  unsigned long long overflow;  // a level of a pass did not fit its queue
  unsigned long long invalid;   // cells of x_avg outside [0, 1]
  unsigned long long pad[3];
};

struct MarchArgs {
  const unsigned long long* skip;  // nonzero *skip: return at once (replays after a stop)
  // grid
  int32_t n, periodic, corr, l_max;
  int32_t level;     // HEALPix level of every input ray (-1: injected rays)
  int32_t spawn;     // 1: input ray r is (src_begin + r/12, pix r%12, s 0, w 0/1)
  int32_t lds_keys_fit;  // 1: line indices (cell >> 3) fit 32 bits (Gamma staged in LDS)
  int32_t refill_min;    // idle lanes that trigger a refill of a wavefront
  int64_t claim;         // rays a wavefront claims at a time
  double h_cm, sigma0, tau_max, s_max, h3;
  double inv_h3;     // 1 / h^3 (the mixed path's FP32 deposit scale)
  double r2split;    // split iff s*s > r2split (this level)
  double sqrt_omega; // sqrt of the pixel solid angle (this level)
  double tau_stop;   // the ray stops once tau >= tau_stop: tau_max for a
                     // monochromatic source; for a spectrum the threshold
                     // optical depth at which Phi(tau) reaches tau_max
  float kf;          // (float)(sigma0 * h_cm)
  int32_t spec_nint;            // polychromatic: table intervals in use
  const SpecRec64* spec64;      // polychromatic table (FP64 path, and ray set-up)
  const SpecRec32* spec32;      // the same for the mixed path
  const double* a64; // absorber, sign bit set = not a usable neighbour
  double* gamma;
  // sources
  const double* dirs;     // HEALPix directions (x, y, z) of levels 0..dir_max_level
  int32_t dir_max_level;
  const double* src_pos;  // 3 per source
  const double* src_l0;   // rate per level-0 ray (ndot / 12)
  int64_t src_begin;
  // input rays [begin, end), or [0, *count_src) when count_src is set (the
  // previous level's kernel wrote the count; at most in_cap)
  int64_t begin, end;
  const unsigned long long* count_src;
  int64_t in_cap;
  unsigned long long* claim_ctr;  // rays claimed so far in this launch
  RayQueue in;
  // injected rays (level == -1)
  const double* inj_origin;
  const double* inj_dir;
  const int32_t* inj_level;
  const double* inj_L;
  double sqrt_omega_tab[kMaxLevel + 1];  // per level, for injected rays
  // output rays (next level)
  RayQueue out;
  int64_t out_cap;
  Accum* acc;
};

// Workspace carve-out (byte offsets into the caller's buffer).
// HEALPix directions of every pixel of levels 0..kDirTableMaxLevel are kept
// in a table (24 B per pixel: 1.6 GB at level 11); deeper levels compute them
constexpr int kDirTableMaxLevel = 11;

// first table entry of a level: 12 (4^0 + ... + 4^(level-1)) = 4 (4^level - 1)
__host__ __device__ inline int64_t dir_table_offset(int level) {
  return 4 * ((int64_t(1) << (2 * level)) - 1);
}

struct Layout {
  size_t n_H, x, a, srcpos, srcl0, srcaux, queues, accum, rt, dirs, spec, scratch, total;
  int64_t cells, max_sources, capacity;
  int levels;      // number of level queues (levels 1..l_max)
  int dir_levels;  // direction table covers levels 0..dir_levels
};

Layout plan_layout(const nrt_grid_desc& d, int64_t max_sources, int64_t capacity);

// march arguments that follow from the grid alone (no sources, queues or
// direction table: the caller sets those); tau_stop is tau_max
MarchArgs march_grid_args(const nrt_grid_desc& d, const double* a64,
                          double* gamma, Accum* acc);

// the reason a grid descriptor is invalid, or NULL (capi.hip)
const char* check_grid_desc(const nrt_grid_desc* d);
// set the message nrt_last_error(NULL) returns (fixed storage, no allocation)
void set_error(const char* msg);

}  // namespace nrt

struct nrt_ctx {
  nrt_grid_desc desc;
  nrt::Layout lay;
  int device;
  int cu_count;
  int march_blocks_per_cu;  // resident blocks of the march kernel per CU
  nrt_tuning tuning;        // launch parameters (0 = default)
  // captured device-driven pass (hipGraph)
  hipGraphExec_t graph_exec;
  hipStream_t capture_stream;
  double* graph_gamma;      // Gamma buffer the graph writes
  int64_t graph_sources;    // source count the graph was captured for
  nrt_tuning graph_tuning;  // launch parameters it was captured with
  bool graph_eligible;      // a previous pass fit every level in one queue
  // captured pass of a radiation step (absorber, trace, chemistry, check)
  hipGraphExec_t rt_exec;
  double rt_key[4];         // dt, alpha, tol, change threshold it was captured with
  int64_t rt_max_iter;
  double* rt_gamma;
  int64_t rt_sources;
  nrt_tuning rt_tuning;
  int last_pass_graph;      // 1 if the last pass replayed the graph
  hipStream_t stream;
  char* ws;
  // typed views into the workspace
  double* n_H;
  double* x;
  double* a64;
  double* dirs;
  nrt::SpecRec64* spec64;
  nrt::SpecRec32* spec32;
  double* spec_nodes;  // m0, mean, variance at the table's nodes
  int32_t spec_nint;
  double spec_tau_stop;  // threshold optical depth where Phi reaches tau_max
  double* src_pos;
  double* src_l0;
  nrt::RayQueue queue[nrt::kMaxLevel + 1];
  nrt::Accum* acc;
  nrt::RtState* rt;
  char* scratch;
  size_t scratch_bytes;
  // host mirror of the source table
  std::vector<double> h_pos, h_ndot, h_radius;
  bool sources_dirty;
  // pinned host staging for small readbacks
  nrt::Accum* h_acc;
  // per-level constants (host-computed, FP64)
  double r2split[nrt::kMaxLevel + 1];
  double sqrt_omega[nrt::kMaxLevel + 1];
  // timing of the last pass
  std::vector<hipEvent_t> ev;
  int launches;
  double march_ms;
  std::string err;
};

namespace nrt {

// trace.hip
hipError_t launch_prep(nrt_ctx* c);
// the same from another ionized fraction, skipped while *skip is nonzero
hipError_t launch_prep_from(nrt_ctx* c, const double* x, const unsigned long long* skip,
                            hipStream_t s);
// absorber from n_H and x, invalid input cells counted in acc->invalid
hipError_t launch_prep_fields(const double* n_H, const double* x, double n_th, int64_t ncell,
                              double* a64, Accum* acc, int cus, hipStream_t s);
// the march on a persistent grid of at most cu_count * resident_per_cu blocks
hipError_t launch_march_on(const nrt_grid_desc& d, int cu_count, int resident_per_cu,
                           const nrt_tuning& t, const MarchArgs& a, int64_t rays,
                           hipStream_t st);
// l0[k] = ndot[k] / 12 on the device
hipError_t launch_source_rates(const double* ndot, int64_t m, double* l0, hipStream_t s);
hipError_t launch_zero(double* p, int64_t count, int cus, hipStream_t s,
                       const unsigned long long* skip = nullptr);
hipError_t launch_zero_accum(Accum* acc, hipStream_t s, const unsigned long long* skip = nullptr);
// end of a captured radiation-step pass: count it, stop the iteration when
// at most `threshold` cells changed, at max_iter passes, or on an overflow or
// invalid input (one thread)
hipError_t launch_rt_check(const Accum* acc, RtState* rt, unsigned long long threshold,
                           unsigned long long max_iter, hipStream_t s);
hipError_t launch_rt_reset(RtState* rt, hipStream_t s);
hipError_t launch_march(const nrt_ctx* c, const MarchArgs& a, int64_t rays, hipStream_t st);
hipError_t march_blocks_per_cu(const nrt_grid_desc& d, int* blocks);
hipError_t launch_healpix(int level, int64_t first, int64_t count, double* out, hipStream_t s);
// the threshold optical depth where a spectrum's Phi reaches tau_max, written
// to one device double (the spectrum table must be built)
hipError_t launch_spec_stop(const nrt_ctx* c, double* out);
// budget of a device-driven pass into device memory: emitted and the spawn
// count come from the host, the rest from the accumulator block
hipError_t launch_budget(const Accum* acc, nrt_budget* out, uint64_t* dropped, double emitted,
                         int64_t spawned, int l_max, hipStream_t s);

// merge.hip
size_t merge_bytes_per_source();
hipError_t run_merge(nrt_ctx* c, const nrt_merge_params& mp, const double* h_ndot, int64_t m,
                     std::vector<double>& out6, std::string& why);

// spectrum.hip: the polychromatic table.  Fills c->spec64 / c->spec32 and
// c->spec_nint; returns NRT_ERR_ARG (with c->err set) for a spectrum whose
// transmitted share does not fall to 1e-6 e^{-tau_max} within the table.
nrt_status build_spectrum_table(nrt_ctx* c);

// chem.hip
hipError_t launch_chem(const nrt_ctx* c, const double* gamma, double dt, double alpha, double tol,
                       double* x_avg, double* x_new, hipStream_t s,
                       const unsigned long long* skip = nullptr);
hipError_t launch_copy(const nrt_ctx* c, const double* src, double* dst);

}  // namespace nrt
