// Source merging on the GPU (Sec. "Source Merging Algorithm", Alg. source_merge).
//
//   1. snap every source to its cell, sort by (cell, input index) and merge
//      same-cell sources by summing rates in input order;
//   2. max_radius: one wavefront per source grows shells r = k dr <= R_max;
//      the shell's samples are the distinct cells floor(centre + r d_q) over
//      the HEALPix directions d_q of `shell_level` (deduplicated with a hash
//      set in LDS); a shell passes iff N_ion / N_tot >= f_req, or, below
//      N_min samples, iff every sample is ionized;
//   3. pairs with min-image d^2 <= (f_ov (r_a + r_b))^2 + eps and r_a, r_b > 0
//      are united in a lock-free union-find (the larger root is hooked under
//      the smaller, so a group's root is its lowest member); candidates come
//      from a uniform binning whose bins are wider than any overlap distance;
//   4. (root, index) pairs are sorted so each group's members are contiguous
//      and in order; one thread per group sums rates, takes the largest
//      radius, forms the flux-weighted centroid with periodic unwrapping
//      relative to the lowest member, rounds it (floor(c + 1/2)), wraps it and
//      snaps it to the nearest member cell (ties: lowest member);
//   5. the merged catalogue is sorted lexicographically by (i, j, k).
// Every decision uses the FP64 operations written here in this order.
#include <algorithm>
#include <cstring>

#include "healpix.h"
#include "internal.h"

namespace nrt {
namespace {

constexpr unsigned long long kPad = ~0ull;

__device__ __forceinline__ int64_t wrap64(int64_t i, int64_t n) {
  const int64_t r = i % n;
  return r < 0 ? r + n : r;
}

__device__ __forceinline__ int64_t min_image(int64_t d, int64_t n, int periodic) {
  if (!periodic) return d;
  d = wrap64(d, n);
  if (2 * d > n) d -= n;
  return d;
}

// ---- bitonic sort of (key, value) pairs, keys compared then values ----
__global__ void k_bitonic(unsigned long long* key, uint32_t* val, int64_t count, int64_t k,
                          int64_t j) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int64_t l = i ^ j;
  if (l <= i) return;
  const unsigned long long ki = key[i], kl = key[l];
  const uint32_t vi = val[i], vl = val[l];
  const bool greater = ki > kl || (ki == kl && vi > vl);
  const bool ascending = (i & k) == 0;
  if (ascending == greater) {
    key[i] = kl;
    key[l] = ki;
    val[i] = vl;
    val[l] = vi;
  }
}

// ---- step 1: keys of the input sources ----
__global__ void k_source_keys(const double* pos, int64_t m, int64_t pow2, int64_t n,
                              unsigned long long* key, uint32_t* val) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= pow2) return;
  if (s < m) {
    const int64_t i = int64_t(floor(pos[3 * s])), j = int64_t(floor(pos[3 * s + 1])),
                  k = int64_t(floor(pos[3 * s + 2]));
    key[s] = static_cast<unsigned long long>((i * n + j) * n + k);
    val[s] = uint32_t(s);
  } else {
    key[s] = kPad;
    val[s] = 0xffffffffu;
  }
}

// head flag of each run of equal keys (sorted)
__global__ void k_run_heads(const unsigned long long* key, int64_t m, uint32_t* flag) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= m) return;
  flag[s] = (s == 0 || key[s] != key[s - 1]) ? 1u : 0u;
}

// exclusive scan, block level: 1024 threads x 1 item; block sums out
__global__ void k_scan_block(const uint32_t* in, uint32_t* out, uint32_t* block_sums,
                             int64_t count) {
  __shared__ uint32_t sh[1024];
  const int64_t i = int64_t(blockIdx.x) * 1024 + threadIdx.x;
  const uint32_t v = i < count ? in[i] : 0u;
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const uint32_t t = threadIdx.x >= unsigned(off) ? sh[threadIdx.x - off] : 0u;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  if (i < count) out[i] = sh[threadIdx.x] - v;
  if (threadIdx.x == 1023) block_sums[blockIdx.x] = sh[1023];
}

__global__ void k_scan_add(uint32_t* out, const uint32_t* block_offsets, int64_t count) {
  const int64_t i = int64_t(blockIdx.x) * 1024 + threadIdx.x;
  if (i < count) out[i] += block_offsets[blockIdx.x];
}

// dedupe: the head of each run sums the run's rates in input order
__global__ void k_dedupe(const unsigned long long* key, const uint32_t* val, const uint32_t* flag,
                         const uint32_t* slot, const double* ndot, int64_t m, int64_t n,
                         int32_t* cells, double* flux) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= m || !flag[s]) return;
  double f = ndot[val[s]];
  for (int64_t t = s + 1; t < m && !flag[t]; ++t) f += ndot[val[t]];
  const int64_t o = slot[s];
  const int64_t kk = int64_t(key[s]);
  cells[3 * o] = int32_t(kk / (n * n));
  cells[3 * o + 1] = int32_t((kk / n) % n);
  cells[3 * o + 2] = int32_t(kk % n);
  flux[o] = f;
}

__global__ void k_shell_dirs(int level, int64_t count, double* dirs) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= count) return;
  double x, y, z;
  healpix_dir(level, uint32_t(q), x, y, z);
  dirs[3 * q] = x;
  dirs[3 * q + 1] = y;
  dirs[3 * q + 2] = z;
}

// ---- step 2: max_radius, one wavefront per source ----
constexpr int kHash = 4096;  // >= 2 x samples per shell (768 at level 3)
constexpr int kWavesPerBlock = 2;

__global__ __launch_bounds__(64 * kWavesPerBlock) void k_max_radius(
    const int32_t* cells, int64_t m, const double* x, int64_t n, int periodic,
    const double* dirs, int nsamp, double dr, double x_th, double f_req, int n_min, double r_max,
    double* radius) {
  __shared__ unsigned long long table[kWavesPerBlock][kHash];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int64_t s = int64_t(blockIdx.x) * kWavesPerBlock + wave;
  if (s >= m) return;  // whole wavefront leaves together
  unsigned long long* tab = table[wave];
  const int64_t ci = cells[3 * s], cj = cells[3 * s + 1], ck = cells[3 * s + 2];
  if (x[ci + n * (cj + n * ck)] < x_th) {
    if (lane == 0) radius[s] = 0.0;
    return;
  }
  double result = r_max;
  for (int64_t kk = 1;; ++kk) {
    const double r = double(kk) * dr;
    if (!(r <= r_max)) break;
    for (int q = lane; q < kHash; q += 64) tab[q] = kPad;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    int ntot = 0, nion = 0;
    for (int q = lane; q < nsamp; q += 64) {
      const double p0 = (double(ci) + 0.5) + r * dirs[3 * q];
      const double p1 = (double(cj) + 0.5) + r * dirs[3 * q + 1];
      const double p2 = (double(ck) + 0.5) + r * dirs[3 * q + 2];
      int64_t v0 = int64_t(floor(p0)), v1 = int64_t(floor(p1)), v2 = int64_t(floor(p2));
      if (periodic) {
        v0 = wrap64(v0, n);
        v1 = wrap64(v1, n);
        v2 = wrap64(v2, n);
      } else if (v0 < 0 || v0 >= n || v1 < 0 || v1 >= n || v2 < 0 || v2 >= n) {
        continue;
      }
      const unsigned long long cell = static_cast<unsigned long long>(v0 + n * (v1 + n * v2));
      unsigned h = unsigned((cell * 0x9E3779B97F4A7C15ull) >> 52) & (kHash - 1);
      for (;;) {
        const unsigned long long prev = atomicCAS(&tab[h], kPad, cell);
        if (prev == kPad) {  // first time this cell is seen
          ++ntot;
          if (x[cell] >= x_th) ++nion;
          break;
        }
        if (prev == cell) break;
        h = (h + 1) & (kHash - 1);
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      ntot += __shfl_xor(ntot, off);
      nion += __shfl_xor(nion, off);
    }
    bool pass;
    if (ntot < n_min)
      pass = (nion == ntot);
    else
      pass = !(double(nion) / double(ntot) < f_req);
    __builtin_amdgcn_wave_barrier();
    if (!pass) {
      result = r - dr;
      break;
    }
  }
  if (lane == 0) radius[s] = result;
}

// ---- step 3: binning and union-find ----
__global__ void k_bin_count(const int32_t* cells, const double* radius, int64_t m, int64_t n,
                            int64_t nb, uint32_t* bin_of, uint32_t* counts) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= m) return;
  if (!(radius[s] > 0.0)) {
    bin_of[s] = 0xffffffffu;
    return;
  }
  const int64_t b = (cells[3 * s] * nb / n) + nb * ((cells[3 * s + 1] * nb / n) +
                                                    nb * (cells[3 * s + 2] * nb / n));
  bin_of[s] = uint32_t(b);
  atomicAdd(&counts[b], 1u);
}

__global__ void k_bin_fill(const uint32_t* bin_of, int64_t m, uint32_t* cursor,
                           uint32_t* members) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= m || bin_of[s] == 0xffffffffu) return;
  const uint32_t p = atomicAdd(&cursor[bin_of[s]], 1u);
  members[p] = uint32_t(s);
}

__device__ int uf_find(int* parent, int a) {
  for (;;) {
    const int p = __hip_atomic_load(&parent[a], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (p == a) return a;
    a = p;
  }
}

__device__ void uf_unite(int* parent, int a, int b) {
  for (;;) {
    a = uf_find(parent, a);
    b = uf_find(parent, b);
    if (a == b) return;
    if (a < b) {
      const int t = a;
      a = b;
      b = t;
    }  // hook the larger root a under the smaller b
    if (atomicCAS(&parent[a], a, b) == a) return;
  }
}

__device__ bool overlaps(const int32_t* ca, const int32_t* cb, double ra, double rb, int64_t n,
                         int periodic, double f_ov, double eps) {
  if (!(ra > 0.0 && rb > 0.0)) return false;
  double d2 = 0.0;
  for (int ax = 0; ax < 3; ++ax) {
    const double dd = double(min_image(int64_t(ca[ax]) - cb[ax], n, periodic));
    d2 += dd * dd;
  }
  const double rsum = f_ov * (ra + rb);
  return d2 <= rsum * rsum + eps;
}

__global__ void k_pairs_binned(const int32_t* cells, const double* radius, const uint32_t* bin_of,
                               const uint32_t* start, const uint32_t* counts,
                               const uint32_t* members, int64_t m, int64_t n, int64_t nb,
                               int periodic, double f_ov, double eps, int* parent) {
  const int64_t a = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (a >= m || bin_of[a] == 0xffffffffu) return;
  const int64_t b0 = bin_of[a];
  const int64_t bx = b0 % nb, by = (b0 / nb) % nb, bz = b0 / (nb * nb);
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        int64_t qx = bx + dx, qy = by + dy, qz = bz + dz;
        if (periodic) {
          qx = wrap64(qx, nb);
          qy = wrap64(qy, nb);
          qz = wrap64(qz, nb);
        } else if (qx < 0 || qx >= nb || qy < 0 || qy >= nb || qz < 0 || qz >= nb) {
          continue;
        }
        const int64_t q = qx + nb * (qy + nb * qz);
        for (uint32_t t = start[q], e = start[q] + counts[q]; t < e; ++t) {
          const int64_t b = members[t];
          if (b > a && overlaps(cells + 3 * a, cells + 3 * b, radius[a], radius[b], n, periodic,
                                f_ov, eps))
            uf_unite(parent, int(a), int(b));
        }
      }
}

__global__ void k_pairs_all(const int32_t* cells, const double* radius, int64_t m, int64_t n,
                            int periodic, double f_ov, double eps, int* parent) {
  const int64_t a = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (a >= m || !(radius[a] > 0.0)) return;
  for (int64_t b = a + 1; b < m; ++b)
    if (overlaps(cells + 3 * a, cells + 3 * b, radius[a], radius[b], n, periodic, f_ov, eps))
      uf_unite(parent, int(a), int(b));
}

__global__ void k_iota(int* parent, int64_t m) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s < m) parent[s] = int(s);
}

// ---- step 4: groups ----
__global__ void k_root_keys(int* parent, int64_t m, int64_t pow2, unsigned long long* key,
                            uint32_t* val) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= pow2) return;
  if (s < m) {
    key[s] = static_cast<unsigned long long>(uf_find(parent, int(s)));
    val[s] = uint32_t(s);
  } else {
    key[s] = kPad;
    val[s] = 0xffffffffu;
  }
}

__global__ void k_collapse(const unsigned long long* root, const uint32_t* member,
                           const uint32_t* flag, const uint32_t* slot, int64_t m,
                           const int32_t* cells, const double* flux, const double* radius,
                           int64_t n, int periodic, int32_t* out_cells, double* out_flux,
                           double* out_radius) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= m || !flag[s]) return;
  int64_t e = s + 1;
  while (e < m && !flag[e]) ++e;
  const int64_t a = member[s];  // lowest member
  const int64_t o = slot[s];
  if (e - s == 1) {
    for (int ax = 0; ax < 3; ++ax) out_cells[3 * o + ax] = cells[3 * a + ax];
    out_flux[o] = flux[a];
    out_radius[o] = radius[a];
    return;
  }
  double ftot = 0.0, rmax = 0.0, cen[3] = {0.0, 0.0, 0.0};
  for (int64_t t = s; t < e; ++t) {
    const int64_t b = member[t];
    ftot += flux[b];
    if (radius[b] > rmax) rmax = radius[b];
    for (int ax = 0; ax < 3; ++ax) {
      const double u = double(int64_t(cells[3 * a + ax]) +
                              min_image(int64_t(cells[3 * b + ax]) - cells[3 * a + ax], n,
                                        periodic));
      cen[ax] += flux[b] * u;
    }
  }
  int64_t rnd[3];
  for (int ax = 0; ax < 3; ++ax) {
    const double cc = cen[ax] / ftot;
    const int64_t v = int64_t(floor(cc + 0.5));
    rnd[ax] = periodic ? wrap64(v, n) : v;
  }
  int64_t best = -1, bestd = 0;
  for (int64_t t = s; t < e; ++t) {
    const int64_t b = member[t];
    int64_t d2 = 0;
    for (int ax = 0; ax < 3; ++ax) {
      const int64_t dd = min_image(int64_t(cells[3 * b + ax]) - rnd[ax], n, periodic);
      d2 += dd * dd;
    }
    if (best < 0 || d2 < bestd) {
      best = b;
      bestd = d2;
    }
  }
  for (int ax = 0; ax < 3; ++ax) out_cells[3 * o + ax] = cells[3 * best + ax];
  out_flux[o] = ftot;
  out_radius[o] = rmax;
  (void)root;
}

// ---- step 5: final order ----
__global__ void k_cell_keys(const int32_t* cells, int64_t m, int64_t pow2, int64_t n,
                            unsigned long long* key, uint32_t* val) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= pow2) return;
  if (s < m) {
    key[s] = static_cast<unsigned long long>((int64_t(cells[3 * s]) * n + cells[3 * s + 1]) * n +
                                             cells[3 * s + 2]);
    val[s] = uint32_t(s);
  } else {
    key[s] = kPad;
    val[s] = 0xffffffffu;
  }
}

__global__ void k_emit(const uint32_t* order, int64_t m, const int32_t* cells, const double* flux,
                       const double* radius, double* out) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= m) return;
  const int64_t g = order[s];
  out[6 * s] = double(cells[3 * g]) + 0.5;
  out[6 * s + 1] = double(cells[3 * g + 1]) + 0.5;
  out[6 * s + 2] = double(cells[3 * g + 2]) + 0.5;
  out[6 * s + 3] = flux[g];
  out[6 * s + 4] = radius[g];
  out[6 * s + 5] = 0.0;
}

unsigned blocks_for(int64_t items, int block) {
  return unsigned(std::max<int64_t>(1, (items + block - 1) / block));
}


static size_t align256z(size_t x) { return (x + 255) & ~size_t(255); }

// exclusive scan of count uint32 values; tmp holds >= 3 (count / 1024 + 16) words
static hipError_t scan_u32(const uint32_t* in, uint32_t* out, int64_t count, uint32_t* tmp,
                           hipStream_t st) {
  const int64_t nb1 = (count + 1023) / 1024;
  hipLaunchKernelGGL(k_scan_block, dim3(unsigned(std::max<int64_t>(nb1, 1))), dim3(1024), 0, st,
                     in, out, tmp, count);
  if (nb1 > 1) {
    uint32_t* sums = tmp;
    uint32_t* offs = tmp + nb1;
    uint32_t* next = offs + nb1;
    hipError_t e = scan_u32(sums, offs, nb1, next, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_add, dim3(unsigned(nb1)), dim3(1024), 0, st, out, offs, count);
  }
  return hipGetLastError();
}

static void bitonic(unsigned long long* key, uint32_t* val, int64_t pow2, hipStream_t st) {
  for (int64_t k = 2; k <= pow2; k <<= 1)
    for (int64_t j = k >> 1; j > 0; j >>= 1)
      hipLaunchKernelGGL(k_bitonic, dim3(blocks_for(pow2, 256)), dim3(256), 0, st, key, val, pow2,
                         k, j);
}

static hipError_t read_count(const uint32_t* slot, const uint32_t* flag, int64_t m,
                             hipStream_t st, int64_t* out) {
  uint32_t v[2] = {0, 0};
  hipError_t e = hipMemcpyAsync(&v[0], slot + m - 1, 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(&v[1], flag + m - 1, 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  *out = int64_t(v[0]) + v[1];
  return e;
}

}  // namespace

size_t merge_bytes_per_source() { return 256; }

// Runs the merge of the context's m sources (positions already on the
// device in src_pos, rates given on the host); out6 receives, per merged
// source in lexicographic order, (x, y, z, rate, radius, 0).
hipError_t run_merge(nrt_ctx* c, const nrt_merge_params& mp, const double* h_ndot, int64_t m,
                     std::vector<double>& out6, std::string& why) {
  const int64_t n = c->desc.n;
  const int periodic = c->desc.periodic;
  hipStream_t st = c->stream;
  int64_t pow2 = 1;
  while (pow2 < m) pow2 <<= 1;
  char* base = c->ws + c->lay.srcaux;
  char* p = base;
  auto take = [&](size_t bytes) {
    char* q = p;
    p += align256z(bytes);
    return q;
  };
  auto* key = reinterpret_cast<unsigned long long*>(take(size_t(pow2) * 8));
  auto* val = reinterpret_cast<uint32_t*>(take(size_t(pow2) * 4));
  auto* flag = reinterpret_cast<uint32_t*>(take(size_t(m) * 4));
  auto* slot = reinterpret_cast<uint32_t*>(take(size_t(m) * 4));
  auto* cells = reinterpret_cast<int32_t*>(take(size_t(m) * 12));
  auto* flux = reinterpret_cast<double*>(take(size_t(m) * 8));
  auto* radius = reinterpret_cast<double*>(take(size_t(m) * 8));
  auto* parent = reinterpret_cast<int*>(take(size_t(m) * 4));
  auto* bin_of = reinterpret_cast<uint32_t*>(take(size_t(m) * 4));
  auto* members = reinterpret_cast<uint32_t*>(take(size_t(m) * 4));
  auto* ocells = reinterpret_cast<int32_t*>(take(size_t(m) * 12));
  auto* oflux = reinterpret_cast<double*>(take(size_t(m) * 8));
  auto* orad = reinterpret_cast<double*>(take(size_t(m) * 8));
  auto* d_ndot = reinterpret_cast<double*>(take(size_t(m) * 8));
  auto* d_out6 = reinterpret_cast<double*>(take(size_t(m) * 48));
  if (size_t(p - base) > size_t(c->lay.max_sources) * merge_bytes_per_source() + 16 * 256) {
    why = "merge scratch exceeds the source area";
    return hipErrorInvalidValue;
  }
  // general scratch: shell directions, scan temporaries, bins
  const int nsamp = 12 << (2 * mp.shell_level);
  const double reach = 2.0 * mp.f_ov * mp.r_max + std::sqrt(std::max(mp.eps, 0.0)) + 1.0;
  int64_t nb = int64_t(std::floor(double(n) / reach));
  if (nb < 3) nb = 1;
  auto scratch_need = [&](int64_t nbins) {
    const int64_t big = std::max(m, nbins);
    return align256z(size_t(nsamp) * 24) + align256z((size_t(big) / 1024 + 16) * 12) +
           3 * align256z(size_t(nbins) * 4);
  };
  while (nb > 1 && scratch_need(nb * nb * nb) > c->scratch_bytes) --nb;
  if (nb < 3) nb = 1;
  if (scratch_need(nb * nb * nb) > c->scratch_bytes) {
    why = "merge scratch exceeds the workspace scratch";
    return hipErrorInvalidValue;
  }
  const int64_t nbin = nb * nb * nb;
  char* g = c->scratch;
  auto gtake = [&](size_t bytes) {
    char* q = g;
    g += align256z(bytes);
    return q;
  };
  auto* dirs = reinterpret_cast<double*>(gtake(size_t(nsamp) * 24));
  auto* scan_tmp = reinterpret_cast<uint32_t*>(gtake((size_t(std::max(m, nbin)) / 1024 + 16) * 12));
  auto* bcount = reinterpret_cast<uint32_t*>(gtake(size_t(nbin) * 4));
  auto* bstart = reinterpret_cast<uint32_t*>(gtake(size_t(nbin) * 4));
  auto* bcursor = reinterpret_cast<uint32_t*>(gtake(size_t(nbin) * 4));

  hipError_t e = hipMemcpyAsync(d_ndot, h_ndot, size_t(m) * 8, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;

  // 1. snap, sort by (cell, input index), merge same-cell sources
  hipLaunchKernelGGL(k_source_keys, dim3(blocks_for(pow2, 256)), dim3(256), 0, st, c->src_pos, m,
                     pow2, n, key, val);
  bitonic(key, val, pow2, st);
  hipLaunchKernelGGL(k_run_heads, dim3(blocks_for(m, 256)), dim3(256), 0, st, key, m, flag);
  if ((e = scan_u32(flag, slot, m, scan_tmp, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_dedupe, dim3(blocks_for(m, 256)), dim3(256), 0, st, key, val, flag, slot,
                     d_ndot, m, n, cells, flux);
  int64_t m1 = 0;
  if ((e = read_count(slot, flag, m, st, &m1)) != hipSuccess) return e;

  // 2. bubble radii
  hipLaunchKernelGGL(k_shell_dirs, dim3(blocks_for(nsamp, 256)), dim3(256), 0, st,
                     mp.shell_level, int64_t(nsamp), dirs);
  hipLaunchKernelGGL(k_max_radius, dim3(blocks_for(m1, kWavesPerBlock)),
                     dim3(64 * kWavesPerBlock), 0, st, cells, m1, c->x, n, periodic, dirs, nsamp,
                     mp.dr, mp.x_th, mp.f_req, mp.n_min, mp.r_max, radius);

  // 3. overlaps and union-find
  hipLaunchKernelGGL(k_iota, dim3(blocks_for(m1, 256)), dim3(256), 0, st, parent, m1);
  if (nb == 1) {
    hipLaunchKernelGGL(k_pairs_all, dim3(blocks_for(m1, 256)), dim3(256), 0, st, cells, radius,
                       m1, n, periodic, mp.f_ov, mp.eps, parent);
  } else {
    if ((e = hipMemsetAsync(bcount, 0, size_t(nbin) * 4, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_bin_count, dim3(blocks_for(m1, 256)), dim3(256), 0, st, cells, radius,
                       m1, n, nb, bin_of, bcount);
    if ((e = scan_u32(bcount, bstart, nbin, scan_tmp, st)) != hipSuccess) return e;
    e = hipMemcpyAsync(bcursor, bstart, size_t(nbin) * 4, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bin_fill, dim3(blocks_for(m1, 256)), dim3(256), 0, st, bin_of, m1,
                       bcursor, members);
    hipLaunchKernelGGL(k_pairs_binned, dim3(blocks_for(m1, 256)), dim3(256), 0, st, cells,
                       radius, bin_of, bstart, bcount, members, m1, n, nb, periodic, mp.f_ov,
                       mp.eps, parent);
  }

  // 4. collapse each group (members contiguous and in order after the sort)
  int64_t pow2b = 1;
  while (pow2b < m1) pow2b <<= 1;
  hipLaunchKernelGGL(k_root_keys, dim3(blocks_for(pow2b, 256)), dim3(256), 0, st, parent, m1,
                     pow2b, key, val);
  bitonic(key, val, pow2b, st);
  hipLaunchKernelGGL(k_run_heads, dim3(blocks_for(m1, 256)), dim3(256), 0, st, key, m1, flag);
  if ((e = scan_u32(flag, slot, m1, scan_tmp, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_collapse, dim3(blocks_for(m1, 256)), dim3(256), 0, st, key, val, flag,
                     slot, m1, cells, flux, radius, n, periodic, ocells, oflux, orad);
  int64_t m2 = 0;
  if ((e = read_count(slot, flag, m1, st, &m2)) != hipSuccess) return e;

  // 5. lexicographic order
  int64_t pow2c = 1;
  while (pow2c < m2) pow2c <<= 1;
  hipLaunchKernelGGL(k_cell_keys, dim3(blocks_for(pow2c, 256)), dim3(256), 0, st, ocells, m2,
                     pow2c, n, key, val);
  bitonic(key, val, pow2c, st);
  hipLaunchKernelGGL(k_emit, dim3(blocks_for(m2, 256)), dim3(256), 0, st, val, m2, ocells, oflux,
                     orad, d_out6);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  out6.resize(size_t(m2) * 6);
  e = hipMemcpyAsync(out6.data(), d_out6, size_t(m2) * 48, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e;
}

}  // namespace nrt
