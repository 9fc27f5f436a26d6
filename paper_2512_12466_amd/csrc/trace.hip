// Ray-tracing kernels for gfx950: absorber preparation and the march.
//
// The march (Alg. trace_rays, Alg. functors) runs one ray per lane.  Rays
// are held in level queues (structure of arrays); a launch takes a range of
// one level's queue, marches every ray until it stops, accumulates the
// photon budget per lane, and appends the four children of every ray that
// splits to the next level's queue.  Children are allocated per wavefront:
// a ballot of the splitting lanes, one atomicAdd by the first of them, and
// each lane's slot from a masked lane count.
//
// Decisions (next cell, split, stop tests, face of the overlap correction)
// are FP64 in both instantiations and use only correctly rounded + - * /
// (the library is compiled with FP contraction off).  MIXED = true computes
// the optical depth, attenuation and deposits in FP32 from an FP32 absorber
// and tracks the transmitted fraction in FP64.
#include <cfloat>
#include <type_traits>

#include "healpix.h"
#include "internal.h"

namespace nrt {

namespace {

__device__ __forceinline__ int wrap_cell(int i, int n) {
  const int r = i % n;
  return r < 0 ? r + n : r;
}

// one step of a wrapped coordinate
__device__ __forceinline__ int wrap_step(int w, int step, int n) {
  w += step;
  if (w >= n) w -= n;
  if (w < 0) w += n;
  return w;
}

// parametric distance from the source to the next plane of one axis
__device__ __forceinline__ double plane_t(double o, double d, int i) {
  if (d > 0.0) return (double(i + 1) - o) / d;
  if (d < 0.0) return (double(i) - o) / d;
  return __builtin_inf();
}

// start cell of a ray at q = o + s d: floor(q), except that an exact integer
// with a negative direction component belongs to the cell below
__device__ __forceinline__ int start_cell(double o, double s, double d) {
  const double q = o + s * d;
  const double f = floor(q);
  int i = int(f);
  if (q == f && d < 0.0) i -= 1;
  return i;
}

__device__ __forceinline__ unsigned lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi(unsigned(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo(unsigned(mask), 0u));
}

__device__ __forceinline__ unsigned long long read_lane64(unsigned long long v, int lane) {
  const unsigned lo = __builtin_amdgcn_readlane(unsigned(v), lane);
  const unsigned hi = __builtin_amdgcn_readlane(unsigned(v >> 32), lane);
  return (static_cast<unsigned long long>(hi) << 32) | lo;
}

struct LaneAcc {
  double absorbed = 0.0, escaped = 0.0, truncated = 0.0;
  unsigned long long segments = 0;
};

// Per-block Gamma accumulator in LDS.  The rays of one block are a bundle of
// neighbouring HEALPix pixels of one source and level (nested pixel order is
// a Z-order curve and children are queued next to each other), so they cross
// the same cells several times; deposits are summed in an open-addressing
// hash table keyed by the cell index and flushed to Gamma with one global
// atomic per distinct cell.  A deposit that finds no slot within kProbe
// probes goes straight to global memory.
constexpr int kSlots = 4096;
constexpr int kProbe = 16;
constexpr uint32_t kEmpty = 0xffffffffu;

template <typename V>
struct DepositTable {
  uint32_t* key;
  V* val;
  double* gamma;
  bool on;  // false when cell indices do not fit 32 bits

  __device__ __forceinline__ void add(int64_t c, V v) const {
    if (on) {
      const uint32_t k = uint32_t(c);
      uint32_t h = (k * 2654435761u) >> (32 - 12);
#pragma unroll 1
      for (int probe = 0; probe < kProbe; ++probe) {
        const uint32_t old = atomicCAS(&key[h], kEmpty, k);
        if (old == kEmpty || old == k) {
          atomicAdd(&val[h], v);
          return;
        }
        h = (h + 1) & (kSlots - 1);
      }
    }
    atomicAdd(gamma + c, double(v));
  }

  // all threads of the block: fold the table into Gamma and clear it
  __device__ __forceinline__ void flush() const {
    __syncthreads();
    for (int q = threadIdx.x; q < kSlots; q += blockDim.x) {
      const uint32_t k = key[q];
      if (k != kEmpty) {
        atomicAdd(gamma + k, double(val[q]));
        key[q] = kEmpty;
        val[q] = V(0);
      }
    }
    __syncthreads();
  }
};

// March one ray from distance s until it stops.  o: source position, d:
// unit direction, L: photon rate of the ray, w: tau (FP64) or exp(-tau)
// (MIXED).  On a split, `split` is set and s_out / w_out carry the state
// the children start from.  Unwrapped cell coordinates (i) keep the plane
// crossings exact across periodic wraps; wrapped ones (w) address memory.
template <bool MIXED>
__device__ void march_ray(const MarchArgs& A, const DepositTable<typename std::conditional<MIXED, float, double>::type>& tab,
                          double o0, double o1, double o2, double d0,
                          double d1, double d2, double L, int level, double r2split,
                          double sqrt_omega, double s, double w, LaneAcc& acc, bool& split,
                          double& s_out, double& w_out) {
  const int n = A.n;
  const int64_t n64 = n;
  const bool open_box = !A.periodic;
  int i0 = start_cell(o0, s, d0), i1 = start_cell(o1, s, d1), i2 = start_cell(o2, s, d2);
  const int st0 = d0 > 0.0 ? 1 : (d0 < 0.0 ? -1 : 0);
  const int st1 = d1 > 0.0 ? 1 : (d1 < 0.0 ? -1 : 0);
  const int st2 = d2 > 0.0 ? 1 : (d2 < 0.0 ? -1 : 0);
  double t0 = plane_t(o0, d0, i0), t1 = plane_t(o1, d1, i1), t2 = plane_t(o2, d2, i2);
  auto outside = [n](int a, int b, int c) {
    return a < 0 || a >= n || b < 0 || b >= n || c < 0 || c >= n;
  };

  // photons carried by the ray: P = L e^{-tau} (FP64), or L * T (MIXED)
  double tau = 0.0, P = 0.0, T = 0.0, absorbed_frac = 0.0;
  float s_rate = 0.0f;  // L / h^3 in FP32 (MIXED)
  if (MIXED) {
    T = w;
    s_rate = float(L / A.h3);
  } else {
    tau = w;
    P = L * exp(-tau);
  }
  if (open_box && outside(i0, i1, i2)) {
    acc.escaped += MIXED ? L * T : P;
    return;
  }
  int w0 = open_box ? i0 : wrap_cell(i0, n);
  int w1 = open_box ? i1 : wrap_cell(i1, n);
  int w2 = open_box ? i2 : wrap_cell(i2, n);

  for (;;) {
    if (A.periodic && s >= A.s_max) {
      acc.escaped += MIXED ? L * T : P;
      break;
    }
    if (MIXED ? (T <= A.t_min) : (tau >= A.tau_max)) {
      acc.truncated += MIXED ? L * T : P;
      break;
    }
    if (s * s > r2split) {
      if (level >= A.l_max) {
        acc.truncated += MIXED ? L * T : P;
        break;
      }
      split = true;
      s_out = s;
      w_out = MIXED ? T : tau;
      break;
    }
    // next crossing: lowest axis wins exact ties
    int ax = 0;
    double tn = t0;
    if (t1 < tn) {
      ax = 1;
      tn = t1;
    }
    if (t2 < tn) {
      ax = 2;
      tn = t2;
    }
    double ds = tn - s;
    if (ds < 0.0) ds = 0.0;
    const int64_t c = int64_t(w0) + n64 * (int64_t(w1) + n64 * int64_t(w2));

    // ---- segment physics (Eq. lut_eqn, Eq. optical_depth) ----
    double G64 = 0.0, a64 = 0.0;
    float G32 = 0.0f, a32 = 0.0f;
    if (MIXED) {
      a32 = fabsf(A.a32[c]);
      const float dsf = float(ds);
      const float dtau = A.kf * a32 * dsf;
      const float em = -expm1f(-dtau);
      const float Tf = float(T);
      const float dT = Tf * em;
      T -= double(dT);
      absorbed_frac += double(dT);
      G32 = a32 > 0.0f ? (s_rate * dT) / a32 : s_rate * Tf * (A.kf * dsf);
    } else {
      a64 = fabs(A.a64[c]);
      const double dl = ds * A.h_cm;
      const double dtau = A.sigma0 * a64 * dl;
      const double dN = P * (-expm1(-dtau));
      G64 = a64 > 0.0 ? dN / (a64 * A.h3) : P * A.sigma0 * dl / A.h3;
      acc.absorbed += dN;
      P -= dN;
      tau += dtau;
    }

    // ---- overlap correction (Eqs. correction .. new_secondary) ----
    double fc = 1.0;
    bool secondary = false;
    int64_t c2 = 0;
    double a2_64 = 0.0;
    float a2_32 = 0.0f;
    if (A.corr != NRT_CORR_NONE) {
      const double rm = 0.5 * (s + tn);
      const double lpix = rm * sqrt_omega;
      // distances from the segment midpoint to the faces of the cell
      double dedge = __builtin_inf();
      int fax = 0, fdir = 1;
      {
        const double m0 = o0 + rm * d0;
        const double dm = m0 - double(i0), dp = double(i0 + 1) - m0;
        const double da = dm < dp ? dm : dp;
        const int sa = dm < dp ? -1 : (dp < dm ? 1 : (d0 < 0.0 ? -1 : 1));
        dedge = da;
        fdir = sa;
      }
      {
        const double m1 = o1 + rm * d1;
        const double dm = m1 - double(i1), dp = double(i1 + 1) - m1;
        const double da = dm < dp ? dm : dp;
        const int sa = dm < dp ? -1 : (dp < dm ? 1 : (d1 < 0.0 ? -1 : 1));
        if (da < dedge) {
          dedge = da;
          fax = 1;
          fdir = sa;
        }
      }
      {
        const double m2 = o2 + rm * d2;
        const double dm = m2 - double(i2), dp = double(i2 + 1) - m2;
        const double da = dm < dp ? dm : dp;
        const int sa = dm < dp ? -1 : (dp < dm ? 1 : (d2 < 0.0 ? -1 : 1));
        if (da < dedge) {
          dedge = da;
          fax = 2;
          fdir = sa;
        }
      }
      if (dedge < 0.5 * lpix) {
        const double f = 0.5 + dedge / lpix;
        if (A.corr == NRT_CORR_LINEAR) {
          fc = f;
        } else if (A.corr == NRT_CORR_SQUARED) {
          fc = f * f;
        } else {
          bool usable = false;
          const int j0 = i0 + (fax == 0 ? fdir : 0);
          const int j1 = i1 + (fax == 1 ? fdir : 0);
          const int j2 = i2 + (fax == 2 ? fdir : 0);
          if (!open_box || !outside(j0, j1, j2)) {
            const int v0 = fax == 0 ? (open_box ? j0 : wrap_step(w0, fdir, n)) : w0;
            const int v1 = fax == 1 ? (open_box ? j1 : wrap_step(w1, fdir, n)) : w1;
            const int v2 = fax == 2 ? (open_box ? j2 : wrap_step(w2, fdir, n)) : w2;
            c2 = int64_t(v0) + n64 * (int64_t(v1) + n64 * int64_t(v2));
            if (MIXED) {
              const float raw = A.a32[c2];
              usable = !__builtin_signbit(raw);
              a2_32 = raw;
            } else {
              const double raw = A.a64[c2];
              usable = !__builtin_signbit(raw);
              a2_64 = raw;
            }
          }
          if (A.corr == NRT_CORR_CONSERVATIVE) {
            if (usable) fc = f;
          } else {  // NAIVE
            fc = f;
          }
          secondary = usable;
        }
      }
    }

    // ---- deposit ----
    if constexpr (MIXED) {
      const float fcf = float(fc);
      tab.add(c, fcf * G32);
      if (secondary) tab.add(c2, ((1.0f - fcf) * (a32 / a2_32)) * G32);
    } else {
      tab.add(c, fc * G64);
      if (secondary) tab.add(c2, ((1.0 - fc) * (a64 / a2_64)) * G64);
    }

    // ---- advance one cell ----
    s = tn;
    if (ax == 0) {
      i0 += st0;
      w0 = open_box ? i0 : wrap_step(w0, st0, n);
      t0 = plane_t(o0, d0, i0);
    } else if (ax == 1) {
      i1 += st1;
      w1 = open_box ? i1 : wrap_step(w1, st1, n);
      t1 = plane_t(o1, d1, i1);
    } else {
      i2 += st2;
      w2 = open_box ? i2 : wrap_step(w2, st2, n);
      t2 = plane_t(o2, d2, i2);
    }
    acc.segments += 1;
    if (open_box && outside(i0, i1, i2)) {
      acc.escaped += MIXED ? L * T : P;
      break;
    }
  }
  if (MIXED) acc.absorbed += L * absorbed_frac;
}

template <bool MIXED>
__global__ __launch_bounds__(kBlock) void k_march(MarchArgs A) {
  using V = typename std::conditional<MIXED, float, double>::type;
  // the deposit table, reused for the budget reduction at the end
  __shared__ __align__(16) unsigned char lds[kSlots * (sizeof(uint32_t) + sizeof(V))];
  uint32_t* lds_key = reinterpret_cast<uint32_t*>(lds);
  V* lds_val = reinterpret_cast<V*>(lds + kSlots * sizeof(uint32_t));
  const DepositTable<V> tab{lds_key, lds_val, A.gamma, A.lds_keys_fit != 0};
  for (int q = threadIdx.x; q < kSlots; q += kBlock) {
    lds_key[q] = kEmpty;
    lds_val[q] = V(0);
  }
  __syncthreads();
  LaneAcc acc;
  const int lane = __lane_id();
  const int64_t stride = int64_t(gridDim.x) * kBlock;
  for (int64_t base = A.begin + int64_t(blockIdx.x) * kBlock; base < A.end; base += stride) {
    const int64_t r = base + threadIdx.x;
    bool split = false;
    uint32_t src = 0, pix = 0;
    double s_out = 0.0, w_out = 0.0;
    if (r < A.end) {
      double o0, o1, o2, d0, d1, d2, L, s, w, r2s, sqo;
      int level;
      if (A.level < 0) {  // injected rays: never split
        o0 = A.inj_origin[3 * r];
        o1 = A.inj_origin[3 * r + 1];
        o2 = A.inj_origin[3 * r + 2];
        d0 = A.inj_dir[3 * r];
        d1 = A.inj_dir[3 * r + 1];
        d2 = A.inj_dir[3 * r + 2];
        L = A.inj_L[r];
        level = A.inj_level[r];
        s = 0.0;
        w = MIXED ? 1.0 : 0.0;
        r2s = __builtin_inf();
        sqo = A.sqrt_omega_tab[level];  // by value in the argument block
      } else {
        if (A.spawn) {
          src = uint32_t(A.src_begin + r / 12);
          pix = uint32_t(r % 12);
          s = 0.0;
          w = MIXED ? 1.0 : 0.0;
        } else {
          src = A.in.src[r];
          pix = A.in.pix[r];
          s = A.in.s[r];
          w = A.in.w[r];
        }
        level = A.level;
        o0 = A.src_pos[3 * int64_t(src)];
        o1 = A.src_pos[3 * int64_t(src) + 1];
        o2 = A.src_pos[3 * int64_t(src) + 2];
        L = ldexp(A.src_l0[src], -2 * level);
        healpix_dir(level, pix, d0, d1, d2);
        r2s = A.r2split;
        sqo = A.sqrt_omega;
      }
      march_ray<MIXED>(A, tab, o0, o1, o2, d0, d1, d2, L, level, r2s, sqo, s, w, acc, split,
                       s_out, w_out);
    }
    tab.flush();
    // children of the rays that split: one allocation per wavefront
    const uint64_t mask = __ballot(split);
    if (mask) {
      const int leader = __builtin_ctzll(mask);
      unsigned long long slot0 = 0;
      if (lane == leader)
        slot0 = atomicAdd(&A.acc->out_count[A.level + 1],
                          4ull * static_cast<unsigned long long>(__popcll(mask)));
      slot0 = read_lane64(slot0, leader);
      if (split) {
        const unsigned long long slot = slot0 + 4ull * lanes_below(mask);
        if (slot + 4 <= static_cast<unsigned long long>(A.out_cap)) {
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            A.out.src[slot + k] = src;
            A.out.pix[slot + k] = 4u * pix + uint32_t(k);
            A.out.s[slot + k] = s_out;
            A.out.w[slot + k] = w_out;
          }
        } else {
          atomicAdd(&A.acc->overflow, 1ull);
        }
      }
    }
  }

  // block reduction of the lane budgets, then one atomic per block and term
  // (the deposit table is empty after its last flush)
  static_assert(kSlots * (sizeof(uint32_t) + sizeof(V)) >= kBlock * 32, "reduction space");
  double(*red_d)[kBlock] = reinterpret_cast<double(*)[kBlock]>(lds);
  unsigned long long* red_u = reinterpret_cast<unsigned long long*>(lds + 3 * kBlock * 8);
  red_d[0][threadIdx.x] = acc.absorbed;
  red_d[1][threadIdx.x] = acc.escaped;
  red_d[2][threadIdx.x] = acc.truncated;
  red_u[threadIdx.x] = acc.segments;
  __syncthreads();
  for (int h = kBlock / 2; h > 0; h >>= 1) {
    if (int(threadIdx.x) < h) {
      red_d[0][threadIdx.x] += red_d[0][threadIdx.x + h];
      red_d[1][threadIdx.x] += red_d[1][threadIdx.x + h];
      red_d[2][threadIdx.x] += red_d[2][threadIdx.x + h];
      red_u[threadIdx.x] += red_u[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd(&A.acc->absorbed, red_d[0][0]);
    atomicAdd(&A.acc->escaped, red_d[1][0]);
    atomicAdd(&A.acc->truncated, red_d[2][0]);
    atomicAdd(&A.acc->segments, red_u[0]);
  }
}

// a = (1 - x) n_H with the neighbour flag in the sign bit: a cell is a
// usable neighbour (Eqs. new_correction / new_secondary) iff n_H >= n_th and
// a > 0; otherwise -a is stored (-0.0 for a = 0).  Invalid inputs are counted.
__global__ void k_prep(const double* __restrict__ n_H, const double* __restrict__ x, double n_th,
                       int64_t ncell, double* a64, float* a32, Accum* acc) {
  unsigned long long bad = 0;
  for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < ncell;
       c += int64_t(gridDim.x) * blockDim.x) {
    const double nh = n_H[c], xx = x[c];
    if (!(nh >= 0.0) || isinf(nh) || !(xx >= 0.0 && xx <= 1.0)) ++bad;
    const double a = (1.0 - xx) * nh;
    const bool usable = nh >= n_th && a > 0.0;
    if (a64) a64[c] = usable ? a : -a;
    if (a32) {
      float af = float(a);
      if (usable && af < FLT_MIN) af = FLT_MIN;
      a32[c] = usable ? af : -af;
    }
  }
  if (bad) atomicAdd(&acc->invalid, bad);
}

__global__ void k_fill_zero(double* p, int64_t count) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = 0.0;
}

__global__ void k_zero_accum(Accum* acc) {
  unsigned long long* p = reinterpret_cast<unsigned long long*>(acc);
  const int words = int(sizeof(Accum) / sizeof(unsigned long long));
  for (int i = threadIdx.x; i < words; i += blockDim.x) p[i] = 0ull;
}

__global__ void k_healpix(int level, int64_t first, int64_t count, double* out) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= count) return;
  double x, y, z;
  healpix_dir(level, uint32_t(first + q), x, y, z);
  out[3 * q] = x;
  out[3 * q + 1] = y;
  out[3 * q + 2] = z;
}

int grid_for(int64_t items, int block, int cap) {
  int64_t g = (items + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return int(g);
}

}  // namespace

hipError_t launch_prep(nrt_ctx* c) {
  const int64_t ncell = c->lay.cells;
  const bool mixed = c->desc.precision == NRT_MIXED;
  hipLaunchKernelGGL(k_prep, dim3(grid_for(ncell, 256, c->cu_count * 16)), dim3(256), 0,
                     c->stream, c->n_H, c->x, c->desc.n_th, ncell, mixed ? nullptr : c->a64,
                     mixed ? c->a32 : nullptr, c->acc);
  return hipGetLastError();
}

hipError_t launch_zero(double* p, int64_t count, int cus, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(count, 256, cus * 16)), dim3(256), 0, s, p,
                     count);
  return hipGetLastError();
}

hipError_t launch_zero_accum(Accum* acc, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_accum, dim3(1), dim3(256), 0, s, acc);
  return hipGetLastError();
}

hipError_t launch_march(const nrt_ctx* c, const MarchArgs& a, int64_t rays) {
  const int blocks = grid_for(rays, kBlock, c->cu_count * 8);
  if (c->desc.precision == NRT_MIXED)
    hipLaunchKernelGGL(k_march<true>, dim3(blocks), dim3(kBlock), 0, c->stream, a);
  else
    hipLaunchKernelGGL(k_march<false>, dim3(blocks), dim3(kBlock), 0, c->stream, a);
  return hipGetLastError();
}

hipError_t launch_healpix(int level, int64_t first, int64_t count, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_healpix, dim3(grid_for(count, 256, 1 << 20)), dim3(256), 0, s, level,
                     first, count, out);
  return hipGetLastError();
}

}  // namespace nrt
