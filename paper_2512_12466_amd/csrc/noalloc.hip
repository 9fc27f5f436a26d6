// The trace pass for callers that cannot allocate: nrt_trace_step_noalloc.
//
// Every device buffer of the pass beyond the caller's inputs and output (the
// absorber, the source table, the level queues, the accumulators) lives in
// one file-scope device array, `scratch`, of kScratchBytes.  Each GPU that
// runs the library holds its own copy until the process ends; the host finds
// its address once per device with hipGetSymbolAddress and passes that
// address to the kernels.  The call allocates nothing: no hipMalloc or
// hipFree, no host heap (the budget is read back into the caller's struct),
// no events.  Calls on one GPU share its array, so calls that overlap on one
// GPU (from several threads or streams) race; each call clears the state it
// reads before its kernels use it.
#include <cmath>
#include <cstring>
#include <mutex>

#include "internal.h"

// the pass's device state (absorber, sources, accumulators, level queues)
static __device__ __align__(256) unsigned char scratch[size_t(64) << 20];

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per device
constexpr int kMaxDevices = 64;

std::mutex g_mu;
void* g_scratch[kMaxDevices];  // device address of `scratch`, per device
int g_cus[kMaxDevices];

// the message goes where nrt_last_error(NULL) finds it
nrt_status fail(nrt_status s, const char* msg) {
  nrt::set_error(msg);
  return s;
}

size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

// Carve-out of the scratch array for a pass: FP64 absorber, source positions
// and level-0 rates, the accumulators and the level queues 1..l_max.
struct Plan {
  size_t a64, pos, l0, acc, queues, total;
};

Plan plan(const nrt_grid_desc& d, int64_t m, int64_t capacity) {
  const size_t cells = size_t(d.n) * d.n * d.n;
  Plan p;
  size_t off = 0;
  p.a64 = off;
  off = up256(off + cells * 8);
  p.pos = off;
  off = up256(off + size_t(m) * 24);
  p.l0 = off;
  off = up256(off + size_t(m) * 8);
  p.acc = off;
  off = up256(off + sizeof(nrt::Accum));
  p.queues = off;
  const size_t per_level = up256(size_t(capacity) * 4) * 2 + up256(size_t(capacity) * 8) * 2;
  off += per_level * size_t(d.l_max);
  p.total = off;
  return p;
}

// The device address of this device's scratch array, looked up once.
nrt_status device_scratch(int dev, char** base, int* cus) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return fail(NRT_ERR_DEVICE, "hipGetSymbolAddress(scratch) failed");
    int n = 0;
    e = hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return fail(NRT_ERR_DEVICE, "device query failed");
    g_scratch[dev] = ptr;
    g_cus[dev] = n;
  }
  *base = static_cast<char*>(g_scratch[dev]);
  *cus = g_cus[dev];
  return NRT_OK;
}

}  // namespace

extern "C" {

nrt_status nrt_trace_step_noalloc(const nrt_grid_desc* desc, const double* n_H,
                                  const double* x_ion, int64_t m, const double* pos,
                                  const double* ndot, int64_t ray_capacity, double* gamma_out,
                                  nrt_budget* budget, void* hip_stream) {
  if (const char* why = nrt::check_grid_desc(desc)) return fail(NRT_ERR_ARG, why);
  if (desc->spectrum != NRT_SPEC_MONO)
    return fail(NRT_ERR_ARG, "nrt_trace_step_noalloc traces monochromatic sources only");
  if (!n_H || !x_ion || !gamma_out || !budget || m < 0 || (m > 0 && (!pos || !ndot)))
    return fail(NRT_ERR_ARG, "NULL field, output or source array");
  if (ray_capacity < 64 || ray_capacity > (int64_t(1) << 32))
    return fail(NRT_ERR_ARG, "ray_capacity must be in [64, 2^32]");
  const double nn = double(desc->n);
  double emitted = 0.0;
  for (int64_t k = 0; k < m; ++k) {
    for (int a = 0; a < 3; ++a)
      if (!(pos[3 * k + a] >= 0.0 && pos[3 * k + a] < nn))
        return fail(NRT_ERR_ARG, "a source lies outside [0, n)");
    if (!(ndot[k] >= 0.0) || !std::isfinite(ndot[k]))
      return fail(NRT_ERR_ARG, "a source has a bad rate");
    emitted += ndot[k];
  }
  static_assert(sizeof(scratch) == kScratchBytes, "scratch size");
  const Plan p = plan(*desc, m, ray_capacity);
  if (p.total > kScratchBytes)
    return fail(NRT_ERR_NOMEM, "grid, sources and ray queues exceed the 64 MiB static scratch");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return fail(NRT_ERR_DEVICE, "no current HIP device");
  char* base = nullptr;
  int cus = 0;
  nrt_status st = device_scratch(dev, &base, &cus);
  if (st) return st;
  int resident = 0;
  if (nrt::march_blocks_per_cu(*desc, &resident) != hipSuccess)
    return fail(NRT_ERR_DEVICE, "occupancy query failed");

  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const int64_t cells = int64_t(desc->n) * desc->n * desc->n;
  double* a64 = reinterpret_cast<double*>(base + p.a64);
  double* src_pos = reinterpret_cast<double*>(base + p.pos);
  double* src_l0 = reinterpret_cast<double*>(base + p.l0);
  nrt::Accum* acc = reinterpret_cast<nrt::Accum*>(base + p.acc);
  nrt::RayQueue q[nrt::kMaxLevel + 2] = {};
  char* qp = base + p.queues;
  const size_t cap = size_t(ray_capacity);
  for (int l = 1; l <= desc->l_max; ++l) {
    q[l].src = reinterpret_cast<uint32_t*>(qp);
    qp += up256(cap * 4);
    q[l].pix = reinterpret_cast<uint32_t*>(qp);
    qp += up256(cap * 4);
    q[l].s = reinterpret_cast<double*>(qp);
    qp += up256(cap * 8);
    q[l].w = reinterpret_cast<double*>(qp);
    qp += up256(cap * 8);
  }
  auto dev_fail = [&](hipError_t e) {
    return fail(NRT_ERR_DEVICE, hipGetErrorString(e));
  };
  hipError_t e = nrt::launch_zero_accum(acc, s);
  if (e == hipSuccess)
    e = nrt::launch_prep_fields(n_H, x_ion, desc->n_th, cells, a64, acc, cus, s);
  if (e == hipSuccess && m > 0)
    e = hipMemcpyAsync(src_pos, pos, size_t(m) * 24, hipMemcpyHostToDevice, s);
  // the rates go into their slot as given and are divided by 12 in place on
  // the device (no host staging buffer)
  if (e == hipSuccess && m > 0)
    e = hipMemcpyAsync(src_l0, ndot, size_t(m) * 8, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = nrt::launch_source_rates(src_l0, m, src_l0, s);
  if (e == hipSuccess) e = nrt::launch_zero(gamma_out, cells, cus, s);
  if (e != hipSuccess) return dev_fail(e);

  // the device-driven pass: one launch per HEALPix level, each reading its
  // ray count from the count the previous level wrote
  const nrt_tuning t = {0, 0, 0, 0};
  for (int level = 0; level <= desc->l_max && m > 0; ++level) {
    nrt::MarchArgs a = nrt::march_grid_args(*desc, a64, gamma_out, acc);
    a.src_pos = src_pos;
    a.src_l0 = src_l0;
    a.level = level;
    a.spawn = level == 0 ? 1 : 0;
    a.begin = 0;
    a.end = level == 0 ? 12 * m : 0;
    a.count_src = level == 0 ? nullptr : &acc->out_count[level];
    a.in_cap = ray_capacity;
    a.in = q[level];
    const double omega = (4.0 * M_PI) / (12.0 * std::ldexp(1.0, 2 * level));
    a.r2split = desc->n_min_ray > 0.0 ? 1.0 / (desc->n_min_ray * omega) : INFINITY;
    a.sqrt_omega = std::sqrt(omega);
    a.claim_ctr = &acc->claim_lv[level];
    if (level < desc->l_max) {
      a.out = q[level + 1];
      a.out_cap = ray_capacity;
    } else {
      a.out = q[level];
      a.out_cap = 0;
    }
    e = nrt::launch_march_on(*desc, cus, resident, t, a, level == 0 ? 12 * m : ray_capacity, s);
    if (e != hipSuccess) return dev_fail(e);
  }
  nrt::Accum h;
  e = hipMemcpyAsync(&h, acc, sizeof(h), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return dev_fail(e);
  if (h.invalid)
    return fail(NRT_ERR_ARG, "n_H < 0, non-finite n_H or x outside [0, 1] in some cells");
  nrt_budget b;
  std::memset(&b, 0, sizeof(b));
  b.emitted = emitted;
  b.absorbed = h.absorbed;
  b.escaped = h.escaped;
  b.truncated = h.truncated;
  b.segments = h.segments;
  for (int l = 0; l <= desc->l_max; ++l) {
    const uint64_t k = l == 0 ? uint64_t(12 * m) : uint64_t(h.out_count[l]);
    b.rays_per_level[l] = k;
    b.rays += k;
    if (l > 0) b.splits += k / 4;
  }
  *budget = b;
  if (h.overflow)
    return fail(NRT_ERR_OVERFLOW, "a HEALPix level did not fit ray_capacity");
  return NRT_OK;
}

}  // extern "C"
