// C ABI of the nyxrt library (include/nyxrt.h): argument checking, the
// workspace plan, and the host orchestration of the trace (level queues
// processed depth-first in chunks that always fit the next level's queue).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <thread>

#include "healpix.h"
#include "internal.h"

using nrt::Accum;
using nrt::Layout;
using nrt::RtState;
using nrt::MarchArgs;
using nrt::RayQueue;

namespace {

// message of the last failure that has no context (fixed storage, so that
// setting it allocates nothing)
thread_local char g_init_error[512];

void set_init_error(const char* msg) {
  std::strncpy(g_init_error, msg, sizeof(g_init_error) - 1);
  g_init_error[sizeof(g_init_error) - 1] = 0;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

nrt_status fail(nrt_ctx* c, nrt_status s, const std::string& msg) {
  if (c)
    c->err = msg;
  else
    set_init_error(msg.c_str());
  return s;
}

nrt_status hip_fail(nrt_ctx* c, hipError_t e, const char* what) {
  return fail(c, NRT_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_OR_FAIL(ctx, expr)                               \
  do {                                                       \
    hipError_t e_ = (expr);                                  \
    if (e_ != hipSuccess) return hip_fail((ctx), e_, #expr); \
  } while (0)

// the reason a grid descriptor is invalid, or NULL
const char* check_desc(const nrt_grid_desc* d) {
  if (!d) return "desc is NULL";
  if (d->n < 1 || d->n > 4096) return "n must be in [1, 4096]";
  if (!(d->h_cm > 0.0) || !std::isfinite(d->h_cm)) return "h_cm must be > 0";
  if (!(d->sigma0 >= 0.0) || !std::isfinite(d->sigma0)) return "sigma0 must be >= 0";
  if (!(d->n_min_ray >= 0.0) || !std::isfinite(d->n_min_ray))
    return "n_min_ray must be >= 0";
  if (d->l_max < 0 || d->l_max > NRT_MAX_LEVEL) return "l_max out of range";
  if (!(d->tau_max > 0.0)) return "tau_max must be > 0";
  if (std::isnan(d->n_th)) return "n_th is NaN";
  if (d->corr < NRT_CORR_NONE || d->corr > NRT_CORR_NAIVE) return "bad corr";
  if (d->precision != NRT_FP64 && d->precision != NRT_MIXED) return "bad precision";
  if (d->periodic != 0 && d->periodic != 1) return "periodic must be 0 or 1";
  if (d->spectrum == NRT_SPEC_BLACKBODY) {
    if (!(d->spec_param >= 1e3 && d->spec_param <= 1e7))
      return "blackbody temperature must be in [1e3, 1e7] K";
  } else if (d->spectrum == NRT_SPEC_POWERLAW) {
    if (!(d->spec_param >= 2.5 && d->spec_param <= 50.0))
      return "power-law index must be in [2.5, 50]";
  } else if (d->spectrum != NRT_SPEC_MONO) {
    return "bad spectrum";
  }
  return nullptr;
}

// Omega(l) = 4 pi / (12 4^l) (Eq. split_criterion); split iff s^2 > 1/(N_min Omega(l))
void level_constants(nrt_ctx* c) {
  for (int l = 0; l <= nrt::kMaxLevel; ++l) {
    const double omega = (4.0 * M_PI) / (12.0 * std::ldexp(1.0, 2 * l));
    c->sqrt_omega[l] = std::sqrt(omega);
    c->r2split[l] = c->desc.n_min_ray > 0.0 ? 1.0 / (c->desc.n_min_ray * omega) : INFINITY;
  }
}

nrt_status sync_read_accum(nrt_ctx* c) {
  HIP_OR_FAIL(c, hipMemcpyAsync(c->h_acc, c->acc, sizeof(Accum), hipMemcpyDeviceToHost,
                                c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  return NRT_OK;
}

nrt_status read_u64(nrt_ctx* c, const unsigned long long* dev, unsigned long long* out) {
  HIP_OR_FAIL(c, hipMemcpyAsync(&c->h_acc->out_count[0], dev, sizeof(unsigned long long),
                                hipMemcpyDeviceToHost, c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  *out = c->h_acc->out_count[0];
  return NRT_OK;
}

nrt_status upload_sources(nrt_ctx* c) {
  if (!c->sources_dirty) return NRT_OK;
  const size_t m = c->h_ndot.size();
  if (m) {
    std::vector<double> l0(m);
    for (size_t k = 0; k < m; ++k) l0[k] = c->h_ndot[k] / 12.0;
    HIP_OR_FAIL(c, hipMemcpyAsync(c->src_pos, c->h_pos.data(), m * 3 * sizeof(double),
                                  hipMemcpyHostToDevice, c->stream));
    HIP_OR_FAIL(c, hipMemcpyAsync(c->src_l0, l0.data(), m * sizeof(double),
                                  hipMemcpyHostToDevice, c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  }
  c->sources_dirty = false;
  return NRT_OK;
}

MarchArgs base_args(const nrt_ctx* c, double* gamma) {
  MarchArgs a = nrt::march_grid_args(c->desc, c->a64, gamma, c->acc);
  a.tau_stop = c->desc.spectrum != NRT_SPEC_MONO ? c->spec_tau_stop : c->desc.tau_max;
  a.src_pos = c->src_pos;
  a.src_l0 = c->src_l0;
  a.dirs = c->dirs;
  a.dir_max_level = c->lay.dir_levels;
  a.spec_nint = c->spec_nint;
  a.spec64 = c->spec64;
  a.spec32 = c->spec32;
  return a;
}

struct PassState {
  nrt_budget* b;
  double* gamma;
};

nrt_status launch_timed(nrt_ctx* c, const MarchArgs& a, int64_t rays) {
  const size_t k = size_t(c->launches) * 2;
  while (c->ev.size() < k + 2) {
    hipEvent_t e;
    HIP_OR_FAIL(c, hipEventCreate(&e));
    c->ev.push_back(e);
  }
  HIP_OR_FAIL(c, hipEventRecord(c->ev[k], c->stream));
  HIP_OR_FAIL(c, nrt::launch_march(c, a, rays, c->stream));
  HIP_OR_FAIL(c, hipEventRecord(c->ev[k + 1], c->stream));
  c->launches += 1;
  return NRT_OK;
}

// March rays [begin, end) of `level` (virtual spawn indices when spawn),
// then, depth first, every level below them.  Chunks hold at most a quarter
// of the queue capacity, so the children of a chunk always fit.
nrt_status process_level(nrt_ctx* c, PassState& ps, int level, bool spawn, int64_t begin,
                         int64_t end) {
  const int64_t cap = c->lay.capacity;
  const int64_t chunk = std::max<int64_t>(1, cap / 4);
  const bool last = level >= c->desc.l_max;
  for (int64_t b = begin; b < end; b += chunk) {
    const int64_t e = std::min(end, b + chunk);
    MarchArgs a = base_args(c, ps.gamma);
    a.level = level;
    a.spawn = spawn ? 1 : 0;
    a.src_begin = 0;
    a.begin = b;
    a.end = e;
    a.in = c->queue[level];
    a.r2split = c->r2split[level];
    a.sqrt_omega = c->sqrt_omega[level];
    a.claim_ctr = &c->acc->claim;
    unsigned long long* cnt = &c->acc->out_count[level + 1];
    if (!last) {
      a.out = c->queue[level + 1];
      a.out_cap = cap;
      HIP_OR_FAIL(c, hipMemsetAsync(cnt, 0, sizeof(unsigned long long), c->stream));
    } else {
      a.out = c->queue[level];
      a.out_cap = 0;
    }
    HIP_OR_FAIL(c, hipMemsetAsync(&c->acc->claim, 0, sizeof(unsigned long long), c->stream));
    nrt_status st = launch_timed(c, a, e - b);
    if (st) return st;
    ps.b->rays_per_level[level] += uint64_t(e - b);
    ps.b->rays += uint64_t(e - b);
    if (!last) {
      unsigned long long k = 0;
      st = read_u64(c, cnt, &k);
      if (st) return st;
      if (int64_t(k) > cap)
        return fail(c, NRT_ERR_OVERFLOW, "ray queue overflow at level " + std::to_string(level + 1));
      ps.b->splits += k / 4;
      if (k > 0) {
        st = process_level(c, ps, level + 1, false, 0, int64_t(k));
        if (st) return st;
      }
    }
  }
  return NRT_OK;
}

nrt_status finish_timing(nrt_ctx* c) {
  double total = 0.0;
  for (int q = 0; q < c->launches; ++q) {
    float ms = 0.0f;
    HIP_OR_FAIL(c, hipEventElapsedTime(&ms, c->ev[2 * q], c->ev[2 * q + 1]));
    total += ms;
  }
  c->march_ms = total;
  return NRT_OK;
}

// One trace pass over the current absorber field into gamma, driven from
// the host: level queues processed depth first in chunks.
nrt_status chunked_pass(nrt_ctx* c, double* gamma, nrt_budget* out) {
  nrt_status st = upload_sources(c);
  if (st) return st;
  nrt_budget b;
  std::memset(&b, 0, sizeof(b));
  for (double v : c->h_ndot) b.emitted += v;
  HIP_OR_FAIL(c, nrt::launch_zero(gamma, c->lay.cells, c->cu_count, c->stream));
  HIP_OR_FAIL(c, nrt::launch_zero_accum(c->acc, c->stream));
  c->launches = 0;
  c->march_ms = 0.0;
  PassState ps{&b, gamma};
  const int64_t m = int64_t(c->h_ndot.size());
  if (m > 0) {
    st = process_level(c, ps, 0, true, 0, 12 * m);
    if (st) return st;
  }
  st = sync_read_accum(c);
  if (st) return st;
  st = finish_timing(c);
  if (st) return st;
  const Accum& h = *c->h_acc;
  if (h.overflow) return fail(c, NRT_ERR_OVERFLOW, "ray queue overflow");
  b.absorbed = h.absorbed;
  b.escaped = h.escaped;
  b.truncated = h.truncated;
  b.segments = h.segments;
  if (out) *out = b;
  return NRT_OK;
}

// Enqueue a device-driven pass on stream st: every level's launch reads its
// ray count from the accumulator block (written by the previous level), so
// the whole pass runs without a host round trip.  Needs every level to fit
// its queue; a launch that cannot store a split sets the overflow flag.
// The level launches of a device-driven pass (gamma and the accumulators
// cleared by the caller).
hipError_t enqueue_levels(nrt_ctx* c, hipStream_t st, double* gamma,
                          const unsigned long long* skip) {
  hipError_t e = hipSuccess;
  const int64_t m = int64_t(c->h_ndot.size());
  const int64_t cap = c->lay.capacity;
  for (int level = 0; level <= c->desc.l_max && e == hipSuccess; ++level) {
    MarchArgs a = base_args(c, gamma);
    a.skip = skip;
    a.level = level;
    a.spawn = level == 0 ? 1 : 0;
    a.begin = 0;
    a.end = level == 0 ? 12 * m : 0;
    a.count_src = level == 0 ? nullptr : &c->acc->out_count[level];
    a.in_cap = cap;
    a.in = c->queue[level];
    a.r2split = c->r2split[level];
    a.sqrt_omega = c->sqrt_omega[level];
    a.claim_ctr = &c->acc->claim_lv[level];
    if (level < c->desc.l_max) {
      a.out = c->queue[level + 1];
      a.out_cap = cap;
    } else {
      a.out = c->queue[level];
      a.out_cap = 0;
    }
    e = nrt::launch_march(c, a, level == 0 ? 12 * m : cap, st);
  }
  return e;
}

hipError_t enqueue_device_pass(nrt_ctx* c, hipStream_t st, double* gamma) {
  hipError_t e = nrt::launch_zero(gamma, c->lay.cells, c->cu_count, st);
  if (e == hipSuccess) e = nrt::launch_zero_accum(c->acc, st);
  if (e == hipSuccess) e = enqueue_levels(c, st, gamma, nullptr);
  return e;
}

nrt_status capture_graph(nrt_ctx* c, double* gamma) {
  if (c->graph_exec) {
    HIP_OR_FAIL(c, hipGraphExecDestroy(c->graph_exec));
    c->graph_exec = nullptr;
  }
  if (!c->capture_stream)
    HIP_OR_FAIL(c, hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
  HIP_OR_FAIL(c, hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal));
  const hipError_t e = enqueue_device_pass(c, c->capture_stream, gamma);
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(c->capture_stream, &g);
  if (e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return hip_fail(c, e, "capture of the device-driven pass");
  }
  if (e2 != hipSuccess) return hip_fail(c, e2, "hipStreamEndCapture");
  const hipError_t e3 = hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e3 != hipSuccess) {
    c->graph_exec = nullptr;
    return hip_fail(c, e3, "hipGraphInstantiate");
  }
  c->graph_gamma = gamma;
  c->graph_sources = int64_t(c->h_ndot.size());
  c->graph_tuning = c->tuning;
  return NRT_OK;
}

// Replay the captured device-driven pass (capturing it first if needed).
// NRT_ERR_OVERFLOW if a level did not fit its queue (Gamma is then invalid).
nrt_status graph_pass(nrt_ctx* c, double* gamma, nrt_budget* out) {
  nrt_status st = upload_sources(c);
  if (st) return st;
  const int64_t m = int64_t(c->h_ndot.size());
  if (!c->graph_exec || c->graph_gamma != gamma || c->graph_sources != m ||
      std::memcmp(&c->graph_tuning, &c->tuning, sizeof(nrt_tuning)) != 0) {
    st = capture_graph(c, gamma);
    if (st) return st;
  }
  while (c->ev.size() < 2) {
    hipEvent_t e;
    HIP_OR_FAIL(c, hipEventCreate(&e));
    c->ev.push_back(e);
  }
  HIP_OR_FAIL(c, hipEventRecord(c->ev[0], c->stream));
  HIP_OR_FAIL(c, hipGraphLaunch(c->graph_exec, c->stream));
  HIP_OR_FAIL(c, hipEventRecord(c->ev[1], c->stream));
  st = sync_read_accum(c);
  if (st) return st;
  float ms = 0.0f;
  HIP_OR_FAIL(c, hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
  c->launches = c->desc.l_max + 1;
  c->march_ms = ms;
  const Accum& h = *c->h_acc;
  if (h.overflow) return fail(c, NRT_ERR_OVERFLOW, "a level did not fit its queue");
  nrt_budget b;
  std::memset(&b, 0, sizeof(b));
  for (double v : c->h_ndot) b.emitted += v;
  b.absorbed = h.absorbed;
  b.escaped = h.escaped;
  b.truncated = h.truncated;
  b.segments = h.segments;
  for (int l = 0; l <= c->desc.l_max; ++l) {
    const uint64_t k = l == 0 ? uint64_t(12 * m) : uint64_t(h.out_count[l]);
    b.rays_per_level[l] = k;
    b.rays += k;
    if (l > 0) b.splits += k / 4;
  }
  if (out) *out = b;
  return NRT_OK;
}

// One trace pass: replay the captured device-driven pass when every level
// is known to fit its queue, else (or after an overflow) the chunked pass.
nrt_status trace_pass(nrt_ctx* c, double* gamma, nrt_budget* out) {
  const int mode = c->tuning.graph;
  const bool sources = !c->h_ndot.empty();
  if (sources && mode != 1 && (mode == 2 || c->graph_eligible)) {
    const nrt_status st = graph_pass(c, gamma, out);
    if (st == NRT_OK) {
      c->last_pass_graph = 1;
      return NRT_OK;
    }
    if (st != NRT_ERR_OVERFLOW) return st;
    c->graph_eligible = false;
  }
  c->last_pass_graph = 0;
  nrt_budget b;
  const nrt_status st = chunked_pass(c, gamma, &b);
  if (st) return st;
  uint64_t widest = 0;
  for (int l = 1; l <= c->desc.l_max; ++l) widest = std::max(widest, b.rays_per_level[l]);
  c->graph_eligible = widest <= uint64_t(c->lay.capacity);
  if (out) *out = b;
  return NRT_OK;
}

// The direction table of levels 0..c->lay.dir_levels, computed on the host
// with the C library's sincos on the pixelisation's correctly rounded
// geometry, and copied once.
nrt_status fill_direction_table(nrt_ctx* c) {
  const int64_t total = nrt::dir_table_offset(c->lay.dir_levels + 1);
  std::vector<double> tab;
  try {
    tab.resize(size_t(total) * 3);
  } catch (const std::bad_alloc&) {
    return fail(c, NRT_ERR_NOMEM, "host memory for the direction table");
  }
  const int nt = int(std::max(1u, std::min(16u, std::thread::hardware_concurrency())));
  auto work = [&](int t) {
    for (int l = 0; l <= c->lay.dir_levels; ++l) {
      const int64_t first = nrt::dir_table_offset(l), npix = 12 * (int64_t(1) << (2 * l));
      const int64_t lo = npix * t / nt, hi = npix * (t + 1) / nt;
      for (int64_t p = lo; p < hi; ++p) {
        double* d = tab.data() + 3 * (first + p);
        const nrt::HpAngle a = nrt::healpix_angle(l, uint32_t(p));
        double ca = 1.0, sa = 0.0;
        if (a.fold >= 2) ::sincos(a.ang, &sa, &ca);
        nrt::healpix_vector(a, ca, sa, d[0], d[1], d[2]);
      }
    }
  };
  std::vector<std::thread> th;
  for (int t = 1; t < nt; ++t) th.emplace_back(work, t);
  work(0);
  for (auto& x : th) x.join();
  HIP_OR_FAIL(c, hipMemcpyAsync(c->dirs, tab.data(), tab.size() * sizeof(double),
                                hipMemcpyHostToDevice, c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  return NRT_OK;
}

nrt_status prep_absorber(nrt_ctx* c, const double* x_field) {
  const double* keep = c->x;
  c->x = const_cast<double*>(x_field);
  HIP_OR_FAIL(c, nrt::launch_zero_accum(c->acc, c->stream));
  hipError_t e = nrt::launch_prep(c);
  c->x = const_cast<double*>(keep);
  if (e != hipSuccess) return hip_fail(c, e, "launch_prep");
  nrt_status st = sync_read_accum(c);
  if (st) return st;
  if (c->h_acc->invalid)
    return fail(c, NRT_ERR_ARG, std::to_string(c->h_acc->invalid) +
                                    " cells with n_H < 0, non-finite n_H or x outside [0,1]");
  return NRT_OK;
}

// Whether the radiation step's passes can replay a captured graph: the
// device-driven pass fits every level (shown by an earlier pass) and the
// tuning allows graphs.
bool rt_graph_usable(const nrt_ctx* c) {
  return !c->h_ndot.empty() && c->tuning.graph != 1 && (c->tuning.graph == 2 || c->graph_eligible);
}

// Capture one pass of a radiation step on the private stream: the absorber
// from x_avg, the device-driven trace into gamma, the chemistry into x_avg
// and x_new, and the convergence check, every kernel skipped once the check
// has stopped the iteration.  Clears are kernels (no memset nodes).
nrt_status capture_rt_graph(nrt_ctx* c, double dt, double alpha, double tol,
                            unsigned long long threshold, int64_t max_iter, double* gamma,
                            double* x_avg, double* x_new) {
  if (c->rt_exec) {
    HIP_OR_FAIL(c, hipGraphExecDestroy(c->rt_exec));
    c->rt_exec = nullptr;
  }
  if (!c->capture_stream)
    HIP_OR_FAIL(c, hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
  const unsigned long long* skip = &c->rt->done;
  HIP_OR_FAIL(c, hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal));
  hipStream_t s = c->capture_stream;
  // the accumulators first: the absorber kernel counts invalid cells there
  hipError_t e = nrt::launch_zero_accum(c->acc, s, skip);
  if (e == hipSuccess) e = nrt::launch_zero(gamma, c->lay.cells, c->cu_count, s, skip);
  if (e == hipSuccess) e = nrt::launch_prep_from(c, x_avg, skip, s);
  if (e == hipSuccess) e = enqueue_levels(c, s, gamma, skip);
  if (e == hipSuccess) e = nrt::launch_chem(c, gamma, dt, alpha, tol, x_avg, x_new, s, skip);
  if (e == hipSuccess) e = nrt::launch_rt_check(c->acc, c->rt, threshold, max_iter, s);
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(s, &g);
  if (e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return hip_fail(c, e, "capture of a radiation-step pass");
  }
  if (e2 != hipSuccess) return hip_fail(c, e2, "hipStreamEndCapture");
  const hipError_t e3 = hipGraphInstantiate(&c->rt_exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e3 != hipSuccess) {
    c->rt_exec = nullptr;
    return hip_fail(c, e3, "hipGraphInstantiate");
  }
  c->rt_key[0] = dt;
  c->rt_key[1] = alpha;
  c->rt_key[2] = tol;
  c->rt_key[3] = double(threshold);
  c->rt_max_iter = max_iter;
  c->rt_gamma = gamma;
  c->rt_sources = int64_t(c->h_ndot.size());
  c->rt_tuning = c->tuning;
  return NRT_OK;
}

// Replay the captured radiation-step pass until its check stops the
// iteration, starting after `done_iters` host-driven passes: batches of 4
// replays, one readback of the step state per batch.  The replays after the
// stop return at once.  NRT_ERR_OVERFLOW if a level outgrew its queue.
nrt_status rt_replay(nrt_ctx* c, double dt, double alpha, double tol, unsigned long long threshold,
                     int32_t max_iter, int32_t done_iters, double* gamma, double* x_avg,
                     double* x_new, nrt_budget* out, int32_t* iters) {
  nrt_status st = upload_sources(c);
  if (st) return st;
  const int64_t left = int64_t(max_iter) - done_iters;
  if (!c->rt_exec || c->rt_key[0] != dt || c->rt_key[1] != alpha || c->rt_key[2] != tol ||
      c->rt_key[3] != double(threshold) || c->rt_max_iter != left || c->rt_gamma != gamma ||
      c->rt_sources != int64_t(c->h_ndot.size()) ||
      std::memcmp(&c->rt_tuning, &c->tuning, sizeof(nrt_tuning)) != 0) {
    st = capture_rt_graph(c, dt, alpha, tol, threshold, left, gamma, x_avg, x_new);
    if (st) return st;
  }
  HIP_OR_FAIL(c, nrt::launch_rt_reset(c->rt, c->stream));
  RtState h;
  for (;;) {
    for (int r = 0; r < 4; ++r) HIP_OR_FAIL(c, hipGraphLaunch(c->rt_exec, c->stream));
    HIP_OR_FAIL(c, hipMemcpyAsync(&c->h_acc->out_count[0], c->rt, sizeof(RtState),
                                  hipMemcpyDeviceToHost, c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    std::memcpy(&h, &c->h_acc->out_count[0], sizeof(RtState));
    if (h.done) break;
  }
  if (h.overflow) return fail(c, NRT_ERR_OVERFLOW, "a level did not fit its queue");
  if (h.invalid) return fail(c, NRT_ERR_INTERNAL, "the iterated ionized fraction left [0, 1]");
  *iters = done_iters + int32_t(h.iters);
  c->last_pass_graph = 1;
  c->launches = 0;  // not timed
  c->march_ms = 0.0;
  // the budget of the last pass is still in the accumulators
  st = sync_read_accum(c);
  if (st) return st;
  const Accum& a = *c->h_acc;
  nrt_budget b;
  std::memset(&b, 0, sizeof(b));
  for (double v : c->h_ndot) b.emitted += v;
  b.absorbed = a.absorbed;
  b.escaped = a.escaped;
  b.truncated = a.truncated;
  b.segments = a.segments;
  const int64_t m = int64_t(c->h_ndot.size());
  for (int l = 0; l <= c->desc.l_max; ++l) {
    const uint64_t k = l == 0 ? uint64_t(12 * m) : uint64_t(a.out_count[l]);
    b.rays_per_level[l] = k;
    b.rays += k;
    if (l > 0) b.splits += k / 4;
  }
  if (out) *out = b;
  return NRT_OK;
}

}  // namespace

namespace nrt {

const char* check_grid_desc(const nrt_grid_desc* d) { return check_desc(d); }

void set_error(const char* msg) { set_init_error(msg); }

MarchArgs march_grid_args(const nrt_grid_desc& d, const double* a64,
                          double* gamma, Accum* acc) {
  MarchArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n = d.n;
  a.periodic = d.periodic;
  a.corr = d.corr;
  a.l_max = d.l_max;
  a.h_cm = d.h_cm;
  a.sigma0 = d.sigma0;
  a.tau_max = d.tau_max;
  a.s_max = d.periodic ? std::sqrt(3.0) * double(d.n) : INFINITY;
  a.h3 = d.h_cm * d.h_cm * d.h_cm;
  a.inv_h3 = 1.0 / a.h3;
  a.tau_stop = d.tau_max;
  a.kf = float(d.sigma0 * d.h_cm);
  a.a64 = a64;
  a.gamma = gamma;
  a.dir_max_level = -1;  // no direction table: directions computed in the march
  for (int l = 0; l <= kMaxLevel; ++l) {
    const double omega = (4.0 * M_PI) / (12.0 * std::ldexp(1.0, 2 * l));
    a.sqrt_omega_tab[l] = std::sqrt(omega);
  }
  a.acc = acc;
  a.lds_keys_fit = ((int64_t(d.n) * d.n * d.n) >> 3 < (int64_t(1) << 32) - 1) ? 1 : 0;
  return a;
}

Layout plan_layout(const nrt_grid_desc& d, int64_t max_sources, int64_t capacity) {
  Layout L;
  std::memset(&L, 0, sizeof(L));
  const int64_t cells = int64_t(d.n) * d.n * d.n;
  L.cells = cells;
  L.max_sources = max_sources;
  L.capacity = capacity;
  L.levels = d.l_max;
  size_t off = 0;
  L.n_H = off;
  off = align256(off + size_t(cells) * 8);
  L.x = off;
  off = align256(off + size_t(cells) * 8);
  // FP64 absorber in both paths: the optical depth that carries the tau_max
  // decision is FP64, and the mixed path rounds the neighbour's absorber to
  // FP32 where it reads it
  L.a = off;
  off = align256(off + size_t(cells) * 8);
  L.srcpos = off;
  off = align256(off + size_t(max_sources) * 24);
  L.srcl0 = off;
  off = align256(off + size_t(max_sources) * 8);
  L.srcaux = off;
  // merge scratch: per-source arrays plus the alignment of its 15 sub-buffers
  off = align256(off + size_t(max_sources) * nrt::merge_bytes_per_source() + 16 * 256);
  L.queues = off;
  const size_t per_level = align256(size_t(capacity) * 4) * 2 + align256(size_t(capacity) * 8) * 2;
  off += per_level * size_t(L.levels);
  L.accum = off;
  off = align256(off + sizeof(Accum));
  L.rt = off;
  off = align256(off + sizeof(RtState));
  L.dir_levels = std::min(d.l_max, nrt::kDirTableMaxLevel);
  L.dirs = off;
  off = align256(off + size_t(nrt::dir_table_offset(L.dir_levels + 1)) * 24);
  L.spec = off;
  if (d.spectrum != NRT_SPEC_MONO)  // node moments, then the FP64 and FP32 records
    off = align256(off + size_t(3 * kSpecNodes) * 8) +
          size_t(kSpecNodes - 1) * (sizeof(SpecRec64) + sizeof(SpecRec32));
  off = align256(off);
  L.scratch = off;
  // x_avg and x_new of the chemistry; also staging for injected rays and
  // direction queries, hence a 4 MiB floor
  off = align256(off + std::max<size_t>(size_t(cells) * 16, size_t(1) << 22));
  L.total = off;
  return L;
}

}  // namespace nrt

extern "C" {

const char* nrt_status_str(nrt_status s) {
  switch (s) {
    case NRT_OK: return "ok";
    case NRT_ERR_ARG: return "invalid argument";
    case NRT_ERR_STATE: return "invalid state";
    case NRT_ERR_NOMEM: return "workspace too small";
    case NRT_ERR_OVERFLOW: return "queue overflow";
    case NRT_ERR_DEVICE: return "HIP error";
    case NRT_ERR_INTERNAL: return "internal error";
  }
  return "unknown status";
}

const char* nrt_last_error(const nrt_ctx* c) {
  return c ? c->err.c_str() : g_init_error;
}

nrt_status nrt_workspace_bytes(const nrt_grid_desc* desc, int64_t max_sources,
                               int64_t ray_capacity, size_t* bytes) {
  if (const char* why = check_desc(desc)) return fail(nullptr, NRT_ERR_ARG, why);
  if (max_sources < 0 || max_sources > (int64_t(1) << 31))
    return fail(nullptr, NRT_ERR_ARG, "max_sources out of range");
  if (ray_capacity < 4096 || ray_capacity > (int64_t(1) << 32))
    return fail(nullptr, NRT_ERR_ARG, "ray_capacity must be in [4096, 2^32]");
  if (!bytes) return fail(nullptr, NRT_ERR_ARG, "bytes is NULL");
  *bytes = nrt::plan_layout(*desc, max_sources, ray_capacity).total;
  return NRT_OK;
}

nrt_status nrt_init_grid(nrt_ctx** out, const nrt_grid_desc* desc, const double* n_H,
                         const double* x_ion, int64_t max_sources, int64_t ray_capacity,
                         void* workspace, size_t ws_bytes, void* hip_stream) {
  if (!out) return fail(nullptr, NRT_ERR_ARG, "out is NULL");
  *out = nullptr;
  size_t need = 0;
  nrt_status st = nrt_workspace_bytes(desc, max_sources, ray_capacity, &need);
  if (st) return st;
  if (!n_H || !x_ion || !workspace) return fail(nullptr, NRT_ERR_ARG, "NULL field or workspace");
  if (reinterpret_cast<uintptr_t>(workspace) % 256)
    return fail(nullptr, NRT_ERR_ARG, "workspace must be 256-byte aligned");
  if (ws_bytes < need)
    return fail(nullptr, NRT_ERR_NOMEM,
                "workspace has " + std::to_string(ws_bytes) + " bytes, needs " +
                    std::to_string(need));
  nrt_ctx* c = new (std::nothrow) nrt_ctx();
  if (!c) return fail(nullptr, NRT_ERR_NOMEM, "host allocation failed");
  c->desc = *desc;
  c->lay = nrt::plan_layout(*desc, max_sources, ray_capacity);
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->ws = static_cast<char*>(workspace);
  auto bail = [&](nrt_status s) {
    set_init_error(c->err.c_str());
    nrt_destroy(c);
    return s;
  };
  hipError_t e = hipGetDevice(&c->device);
  if (e == hipSuccess)
    e = hipDeviceGetAttribute(&c->cu_count, hipDeviceAttributeMultiprocessorCount, c->device);
  if (e == hipSuccess)
    e = nrt::march_blocks_per_cu(*desc, &c->march_blocks_per_cu);
  if (e != hipSuccess) return bail(hip_fail(c, e, "device query"));
  const Layout& L = c->lay;
  c->n_H = reinterpret_cast<double*>(c->ws + L.n_H);
  c->x = reinterpret_cast<double*>(c->ws + L.x);
  c->a64 = reinterpret_cast<double*>(c->ws + L.a);
  c->src_pos = reinterpret_cast<double*>(c->ws + L.srcpos);
  c->src_l0 = reinterpret_cast<double*>(c->ws + L.srcl0);
  c->dirs = reinterpret_cast<double*>(c->ws + L.dirs);
  if (desc->spectrum != NRT_SPEC_MONO) {
    c->spec_nodes = reinterpret_cast<double*>(c->ws + L.spec);
    c->spec64 = reinterpret_cast<nrt::SpecRec64*>(c->ws + align256(L.spec + 3 * nrt::kSpecNodes * 8));
    c->spec32 = reinterpret_cast<nrt::SpecRec32*>(c->spec64 + (nrt::kSpecNodes - 1));
  }
  char* q = c->ws + L.queues;
  const size_t cap = size_t(L.capacity);
  for (int l = 0; l <= nrt::kMaxLevel; ++l) c->queue[l] = RayQueue{nullptr, nullptr, nullptr, nullptr};
  for (int l = 1; l <= L.levels; ++l) {
    RayQueue& r = c->queue[l];
    r.src = reinterpret_cast<uint32_t*>(q);
    q += align256(cap * 4);
    r.pix = reinterpret_cast<uint32_t*>(q);
    q += align256(cap * 4);
    r.s = reinterpret_cast<double*>(q);
    q += align256(cap * 8);
    r.w = reinterpret_cast<double*>(q);
    q += align256(cap * 8);
  }
  c->acc = reinterpret_cast<Accum*>(c->ws + L.accum);
  c->rt = reinterpret_cast<nrt::RtState*>(c->ws + L.rt);
  c->scratch = c->ws + L.scratch;
  c->scratch_bytes = L.total - L.scratch;
  c->sources_dirty = true;
  level_constants(c);
  e = hipHostMalloc(reinterpret_cast<void**>(&c->h_acc), sizeof(Accum), hipHostMallocDefault);
  if (e != hipSuccess) {
    c->h_acc = nullptr;
    return bail(hip_fail(c, e, "hipHostMalloc"));
  }
  const size_t fb = size_t(L.cells) * sizeof(double);
  e = hipMemcpyAsync(c->n_H, n_H, fb, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(c->x, x_ion, fb, hipMemcpyDeviceToDevice, c->stream);
  if (e != hipSuccess) return bail(hip_fail(c, e, "field copy"));
  st = prep_absorber(c, c->x);
  if (st) return bail(st);
  st = fill_direction_table(c);
  if (st) return bail(st);
  if (desc->spectrum != NRT_SPEC_MONO) {
    st = nrt::build_spectrum_table(c);
    if (st) return bail(st);
    double* stop = reinterpret_cast<double*>(c->scratch);
    e = nrt::launch_spec_stop(c, stop);
    if (e == hipSuccess)
      e = hipMemcpyAsync(&c->h_acc->absorbed, stop, sizeof(double), hipMemcpyDeviceToHost,
                         c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return bail(hip_fail(c, e, "spectrum stop depth"));
    c->spec_tau_stop = c->h_acc->absorbed;
  }
  *out = c;
  return NRT_OK;
}

nrt_status nrt_set_ionization(nrt_ctx* c, const double* x_ion) {
  if (!c) return fail(nullptr, NRT_ERR_ARG, "ctx is NULL");
  if (!x_ion) return fail(c, NRT_ERR_ARG, "x_ion is NULL");
  double* xs = reinterpret_cast<double*>(c->scratch);
  const size_t fb = size_t(c->lay.cells) * sizeof(double);
  // validate on a scratch copy so that a rejected field leaves the context as it was
  HIP_OR_FAIL(c, hipMemcpyAsync(xs, x_ion, fb, hipMemcpyDeviceToDevice, c->stream));
  nrt_status st = prep_absorber(c, xs);
  if (st) {
    prep_absorber(c, c->x);
    return st;
  }
  HIP_OR_FAIL(c, hipMemcpyAsync(c->x, xs, fb, hipMemcpyDeviceToDevice, c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  return NRT_OK;
}

nrt_status nrt_get_ionization(nrt_ctx* c, double* x_out) {
  if (!c) return fail(nullptr, NRT_ERR_ARG, "ctx is NULL");
  if (!x_out) return fail(c, NRT_ERR_ARG, "x_out is NULL");
  HIP_OR_FAIL(c, hipMemcpyAsync(x_out, c->x, size_t(c->lay.cells) * sizeof(double),
                                hipMemcpyDeviceToDevice, c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  return NRT_OK;
}

nrt_status nrt_add_sources(nrt_ctx* c, int64_t m, const double* pos, const double* ndot) {
  if (!c) return fail(nullptr, NRT_ERR_ARG, "ctx is NULL");
  if (m < 0 || (m > 0 && (!pos || !ndot))) return fail(c, NRT_ERR_ARG, "bad source arrays");
  const double n = double(c->desc.n);
  for (int64_t k = 0; k < m; ++k) {
    for (int a = 0; a < 3; ++a) {
      const double p = pos[3 * k + a];
      if (!(p >= 0.0 && p < n))
        return fail(c, NRT_ERR_ARG, "source " + std::to_string(k) + " outside [0, n)");
    }
    if (!(ndot[k] >= 0.0) || !std::isfinite(ndot[k]))
      return fail(c, NRT_ERR_ARG, "source " + std::to_string(k) + " has a bad rate");
  }
  if (int64_t(c->h_ndot.size()) + m > c->lay.max_sources)
    return fail(c, NRT_ERR_OVERFLOW, "source table full");
  c->h_pos.insert(c->h_pos.end(), pos, pos + 3 * m);
  c->h_ndot.insert(c->h_ndot.end(), ndot, ndot + m);
  c->h_radius.insert(c->h_radius.end(), size_t(m), 0.0);
  c->sources_dirty = true;
  return NRT_OK;
}

nrt_status nrt_clear_sources(nrt_ctx* c) {
  if (!c) return fail(nullptr, NRT_ERR_ARG, "ctx is NULL");
  c->h_pos.clear();
  c->h_ndot.clear();
  c->h_radius.clear();
  c->sources_dirty = true;
  return NRT_OK;
}

nrt_status nrt_source_count(const nrt_ctx* c, int64_t* m) {
  if (!c || !m) return fail(const_cast<nrt_ctx*>(c), NRT_ERR_ARG, "NULL argument");
  *m = int64_t(c->h_ndot.size());
  return NRT_OK;
}

nrt_status nrt_get_sources(nrt_ctx* c, double* pos, double* ndot, double* radius) {
  if (!c) return fail(nullptr, NRT_ERR_ARG, "ctx is NULL");
  if (pos) std::copy(c->h_pos.begin(), c->h_pos.end(), pos);
  if (ndot) std::copy(c->h_ndot.begin(), c->h_ndot.end(), ndot);
  if (radius) std::copy(c->h_radius.begin(), c->h_radius.end(), radius);
  return NRT_OK;
}

nrt_status nrt_trace_step(nrt_ctx* c, double* gamma_out, nrt_budget* budget) {
  if (!c) return fail(nullptr, NRT_ERR_ARG, "ctx is NULL");
  if (!gamma_out || !budget) return fail(c, NRT_ERR_ARG, "NULL gamma_out or budget");
  return trace_pass(c, gamma_out, budget);
}

nrt_status nrt_trace_step_async(nrt_ctx* c, double* gamma_out, nrt_budget* budget_dev,
                                uint64_t* dropped_dev) {
  if (!c) return fail(nullptr, NRT_ERR_ARG, "ctx is NULL");
  if (!gamma_out || !budget_dev) return fail(c, NRT_ERR_ARG, "NULL gamma_out or budget_dev");
  if (c->sources_dirty) {  // the table upload copies from host memory and synchronises
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_OR_FAIL(c, hipStreamIsCapturing(c->stream, &cs));
    if (cs != hipStreamCaptureStatusNone)
      return fail(c, NRT_ERR_STATE,
                  "the source table changed since the last pass: run one pass outside stream "
                  "capture first");
    const nrt_status st = upload_sources(c);
    if (st) return st;
  }
  double emitted = 0.0;
  for (double v : c->h_ndot) emitted += v;
  HIP_OR_FAIL(c, enqueue_device_pass(c, c->stream, gamma_out));
  HIP_OR_FAIL(c, nrt::launch_budget(c->acc, budget_dev, dropped_dev, emitted,
                                    12 * int64_t(c->h_ndot.size()), c->desc.l_max, c->stream));
  c->last_pass_graph = 0;
  c->launches = 0;  // not timed
  c->march_ms = 0.0;
  return NRT_OK;
}

nrt_status nrt_trace_rays_debug(nrt_ctx* c, int64_t k, const double* origin, const double* dir,
                                const int32_t* level, const double* L, double* gamma_out,
                                nrt_budget* budget) {
  if (!c) return fail(nullptr, NRT_ERR_ARG, "ctx is NULL");
  if (c->desc.n_min_ray != 0.0) return fail(c, NRT_ERR_STATE, "injected rays need n_min_ray = 0");
  if (k < 0 || (k > 0 && (!origin || !dir || !level || !L)) || !gamma_out || !budget)
    return fail(c, NRT_ERR_ARG, "bad injected-ray arguments");
  const size_t need = size_t(k) * 64;
  if (need > c->scratch_bytes) return fail(c, NRT_ERR_NOMEM, "too many injected rays");
  for (int64_t r = 0; r < k; ++r) {
    for (int a = 0; a < 3; ++a)
      if (!(origin[3 * r + a] >= 0.0 && origin[3 * r + a] < double(c->desc.n)))
        return fail(c, NRT_ERR_ARG, "injected ray origin outside the box");
    if (level[r] < 0 || level[r] > NRT_MAX_LEVEL || !(L[r] >= 0.0) || !std::isfinite(L[r]))
      return fail(c, NRT_ERR_ARG, "bad injected ray level or rate");
    // a direction must be a finite unit vector, or the march would not end
    const double d0 = dir[3 * r], d1 = dir[3 * r + 1], d2 = dir[3 * r + 2];
    const double nn = d0 * d0 + d1 * d1 + d2 * d2;
    if (!std::isfinite(d0) || !std::isfinite(d1) || !std::isfinite(d2) || !(std::fabs(nn - 1.0) <= 1e-9))
      return fail(c, NRT_ERR_ARG, "injected ray direction is not a unit vector");
  }
  double* d_org = reinterpret_cast<double*>(c->scratch);
  double* d_dir = d_org + 3 * k;
  double* d_L = d_dir + 3 * k;
  int32_t* d_lev = reinterpret_cast<int32_t*>(d_L + k);
  HIP_OR_FAIL(c, hipMemcpyAsync(d_org, origin, k * 24, hipMemcpyHostToDevice, c->stream));
  HIP_OR_FAIL(c, hipMemcpyAsync(d_dir, dir, k * 24, hipMemcpyHostToDevice, c->stream));
  HIP_OR_FAIL(c, hipMemcpyAsync(d_L, L, k * 8, hipMemcpyHostToDevice, c->stream));
  HIP_OR_FAIL(c, hipMemcpyAsync(d_lev, level, k * 4, hipMemcpyHostToDevice, c->stream));
  nrt_budget b;
  std::memset(&b, 0, sizeof(b));
  for (int64_t r = 0; r < k; ++r) {
    b.emitted += L[r];
    b.rays_per_level[level[r]] += 1;
  }
  b.rays = uint64_t(k);
  HIP_OR_FAIL(c, nrt::launch_zero(gamma_out, c->lay.cells, c->cu_count, c->stream));
  HIP_OR_FAIL(c, nrt::launch_zero_accum(c->acc, c->stream));
  c->launches = 0;
  if (k > 0) {
    MarchArgs a = base_args(c, gamma_out);
    a.level = -1;
    a.begin = 0;
    a.end = k;
    a.inj_origin = d_org;
    a.inj_dir = d_dir;
    a.inj_L = d_L;
    a.inj_level = d_lev;
    a.out_cap = 0;
    a.claim_ctr = &c->acc->claim;
    HIP_OR_FAIL(c, hipMemsetAsync(&c->acc->claim, 0, sizeof(unsigned long long), c->stream));
    nrt_status st = launch_timed(c, a, k);
    if (st) return st;
  }
  nrt_status st = sync_read_accum(c);
  if (st) return st;
  st = finish_timing(c);
  if (st) return st;
  b.absorbed = c->h_acc->absorbed;
  b.escaped = c->h_acc->escaped;
  b.truncated = c->h_acc->truncated;
  b.segments = c->h_acc->segments;
  *budget = b;
  return NRT_OK;
}

nrt_status nrt_healpix_dirs(nrt_ctx* c, int32_t level, int64_t first, int64_t count,
                            double* out) {
  if (!c) return fail(nullptr, NRT_ERR_ARG, "ctx is NULL");
  const int64_t npix = 12 * (int64_t(1) << (2 * std::max(0, level)));
  if (level < 0 || level > NRT_MAX_LEVEL || first < 0 || count < 0 || first + count > npix ||
      (count > 0 && !out))
    return fail(c, NRT_ERR_ARG, "bad HEALPix range");
  if (count == 0) return NRT_OK;
  // levels in the context's table are read from it (the march's values);
  // deeper levels are computed by the march's device function into scratch
  const double* d = reinterpret_cast<double*>(c->scratch);
  if (level <= c->lay.dir_levels) {
    d = c->dirs + 3 * (nrt::dir_table_offset(level) + first);
  } else {
    if (size_t(count) * 24 > c->scratch_bytes) return fail(c, NRT_ERR_NOMEM, "range too large");
    HIP_OR_FAIL(c, nrt::launch_healpix(level, first, count, reinterpret_cast<double*>(c->scratch),
                                       c->stream));
  }
  HIP_OR_FAIL(c, hipMemcpyAsync(out, d, size_t(count) * 24, hipMemcpyDeviceToHost, c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  return NRT_OK;
}

nrt_status nrt_rt_step(nrt_ctx* c, double dt_s, double alpha, double tol, double conv_frac,
                       int32_t max_iter, double* gamma_out, nrt_budget* budget, int32_t* iters) {
  if (!c) return fail(nullptr, NRT_ERR_ARG, "ctx is NULL");
  if (!(dt_s > 0.0) || !(alpha >= 0.0) || !(tol >= 0.0) || !(conv_frac >= 0.0) ||
      !(conv_frac <= 1.0) || max_iter < 1 || !gamma_out || !budget)
    return fail(c, NRT_ERR_ARG, "bad rt_step arguments");
  double* x_avg = reinterpret_cast<double*>(c->scratch);
  double* x_new = x_avg + c->lay.cells;
  // stop once at most this many cells changed x_avg by tol or more
  const unsigned long long threshold =
      (unsigned long long)std::floor(conv_frac * double(c->lay.cells));
  // one host-driven pass: absorber from x_avg, trace, chemistry, readback;
  // true when the iteration stops after it
  int32_t it = 0;
  auto host_pass = [&](nrt_status& st) {
    ++it;
    st = prep_absorber(c, x_avg);
    if (!st) st = trace_pass(c, gamma_out, budget);
    if (!st) {
      hipError_t e = hipMemsetAsync(&c->acc->chem_changed, 0, sizeof(unsigned long long),
                                    c->stream);
      if (e == hipSuccess)
        e = nrt::launch_chem(c, gamma_out, dt_s, alpha, tol, x_avg, x_new, c->stream);
      st = e == hipSuccess ? sync_read_accum(c) : hip_fail(c, e, "chemistry");
    }
    return st || c->h_acc->chem_changed <= threshold || it >= max_iter;
  };
  nrt_status st = NRT_OK;
  HIP_OR_FAIL(c, nrt::launch_copy(c, c->x, x_avg));
  // the first pass, and every pass while the levels do not fit the queues,
  // is host-driven; then the captured pass (absorber, trace, chemistry and
  // the convergence check on the device) is replayed with one readback per
  // batch of replays
  bool done = host_pass(st);
  while (!done && !rt_graph_usable(c)) done = host_pass(st);
  if (!done) {
    st = rt_replay(c, dt_s, alpha, tol, threshold, max_iter, it, gamma_out, x_avg, x_new, budget,
                   &it);
    if (st == NRT_ERR_OVERFLOW) {  // a level outgrew its queue: redo the step host-driven
      c->graph_eligible = false;
      HIP_OR_FAIL(c, nrt::launch_copy(c, c->x, x_avg));
      it = 0;
      st = NRT_OK;
      while (!host_pass(st)) {
      }
    }
  }
  if (st) {
    prep_absorber(c, c->x);
    return st;
  }
  HIP_OR_FAIL(c, nrt::launch_copy(c, x_new, c->x));
  st = prep_absorber(c, c->x);
  if (st) return st;
  if (iters) *iters = it;
  return NRT_OK;
}

nrt_status nrt_merge_sources(nrt_ctx* c, const nrt_merge_params* mp, int64_t* m_after) {
  if (!c) return fail(nullptr, NRT_ERR_ARG, "ctx is NULL");
  if (!mp || !m_after) return fail(c, NRT_ERR_ARG, "NULL merge parameters or m_after");
  if (!(mp->dr > 0.0) || !std::isfinite(mp->dr) || std::isnan(mp->x_th) ||
      !std::isfinite(mp->f_req) || mp->n_min < 0 || !(mp->r_max >= 0.0) ||
      !std::isfinite(mp->r_max) || !(mp->f_ov >= 0.0) || !std::isfinite(mp->f_ov) ||
      !(mp->eps >= 0.0) || !std::isfinite(mp->eps) || mp->shell_level < 0 ||
      mp->shell_level > 3)
    return fail(c, NRT_ERR_ARG, "bad merge parameters (shell_level must be 0..3)");
  const int64_t m = int64_t(c->h_ndot.size());
  if (m == 0) {
    *m_after = 0;
    return NRT_OK;
  }
  nrt_status st = upload_sources(c);
  if (st) return st;
  std::vector<double> out6;
  std::string why;
  hipError_t e = nrt::run_merge(c, *mp, c->h_ndot.data(), m, out6, why);
  if (e != hipSuccess)
    return why.empty() ? hip_fail(c, e, "source merge") : fail(c, NRT_ERR_NOMEM, why);
  const size_t m2 = out6.size() / 6;
  c->h_pos.resize(3 * m2);
  c->h_ndot.resize(m2);
  c->h_radius.resize(m2);
  for (size_t k = 0; k < m2; ++k) {
    for (int a = 0; a < 3; ++a) c->h_pos[3 * k + a] = out6[6 * k + a];
    c->h_ndot[k] = out6[6 * k + 3];
    c->h_radius[k] = out6[6 * k + 4];
  }
  c->sources_dirty = true;
  *m_after = int64_t(m2);
  return NRT_OK;
}

nrt_status nrt_set_tuning(nrt_ctx* c, const nrt_tuning* t) {
  if (!c) return fail(nullptr, NRT_ERR_ARG, "ctx is NULL");
  if (!t) return fail(c, NRT_ERR_ARG, "tuning is NULL");
  if (t->refill_min < 0 || t->refill_min > 64 || t->claim < 0 || t->claim > 65536 ||
      t->claim % 64 != 0 || t->blocks_per_cu < 0 || t->blocks_per_cu > 64 || t->graph < 0 ||
      t->graph > 2)
    return fail(c, NRT_ERR_ARG, "tuning out of range");
  c->tuning = *t;
  return NRT_OK;
}

nrt_status nrt_get_tuning(const nrt_ctx* c, nrt_tuning* t) {
  if (!c || !t) return fail(const_cast<nrt_ctx*>(c), NRT_ERR_ARG, "NULL argument");
  *t = c->tuning;
  return NRT_OK;
}

nrt_status nrt_autotune(nrt_ctx* c, double* gamma_scratch, int32_t passes, nrt_tuning* best) {
  if (!c) return fail(nullptr, NRT_ERR_ARG, "ctx is NULL");
  if (!gamma_scratch || !best || passes < 1) return fail(c, NRT_ERR_ARG, "bad autotune arguments");
  const nrt_tuning keep = c->tuning;
  std::vector<nrt_tuning> cand;
  const int max_bpc = std::max(1, c->march_blocks_per_cu);
  // refill 64: a wavefront refills only once drained (the best choice where
  // the rays of a run live equally long)
  for (int refill : {8, 16, 32, 64})
    for (int claim : {0, 64, 256})
      for (int bpc : {0, std::max(1, max_bpc - 1)}) {
        if (bpc != 0 && bpc == max_bpc) continue;
        cand.push_back(nrt_tuning{refill, claim, bpc, keep.graph});
      }
  double best_ms = INFINITY;
  nrt_tuning win = keep;
  for (const nrt_tuning& t : cand) {
    c->tuning = t;
    double ms = 0.0;
    for (int p = 0; p < passes; ++p) {
      nrt_budget b;
      nrt_status st = trace_pass(c, gamma_scratch, &b);
      if (st) {
        c->tuning = keep;
        return st;
      }
      ms += c->march_ms;
    }
    if (ms < best_ms) {
      best_ms = ms;
      win = t;
    }
  }
  c->tuning = win;
  *best = win;
  return NRT_OK;
}

nrt_status nrt_last_kernel_time(const nrt_ctx* c, double* march_ms, int32_t* launches,
                                int32_t* graph_replayed) {
  if (!c) return fail(nullptr, NRT_ERR_ARG, "ctx is NULL");
  if (march_ms) *march_ms = c->launches ? c->march_ms / c->launches : 0.0;
  if (launches) *launches = c->launches;
  if (graph_replayed) *graph_replayed = c->last_pass_graph;
  return NRT_OK;
}

nrt_status nrt_destroy(nrt_ctx* c) {
  if (!c) return NRT_OK;
  (void)hipStreamSynchronize(c->stream);
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->rt_exec) (void)hipGraphExecDestroy(c->rt_exec);
  if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  if (c->h_acc) (void)hipHostFree(c->h_acc);
  delete c;
  return NRT_OK;
}

}  // extern "C"
