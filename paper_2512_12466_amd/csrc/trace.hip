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
// are FP64 in both precisions and use only correctly rounded + - * / (the
// library is compiled with FP contraction off).  The optical depth that the
// tau_max stop reads is one of them: both precisions accumulate it in FP64
// from the FP64 absorber by the same operations, so the two paths march the
// same segments and split the same rays.  MIXED = true computes the
// attenuation, the deposits and the correction factors in FP32 (the
// neighbour's absorber rounded from its FP64 word) and tracks the
// transmitted fraction in FP64.  POLY = true integrates the flux
// over a source spectrum with the table of Phi(tau) = -ln F(tau) built at
// context set-up (spectrum.hip).  The march is instantiated per precision,
// correction mode, boundary and spectrum.
#include <cfloat>
#include <cmath>
#include <type_traits>

#include "healpix.h"
#include "internal.h"

namespace nrt {

namespace {

__device__ __forceinline__ int wrap_cell(int i, int n) {
  // start cells lie within a few box lengths of the box: conditional steps
  // instead of an integer division
  if (i >= -2 * n && i < 3 * n) {
    int r = i < 0 ? i + n : i;
    r = r < 0 ? r + n : r;
    r = r >= n ? r - n : r;
    return r >= n ? r - n : r;
  }
  const int r = i % n;
  return r < 0 ? r + n : r;
}

// Flat index of the wrapped cell (w0, w1, w2), x fastest.  n <= 4096, so the
// plane index w1 + n w2 fits 24 bits and one 32 x 32 -> 64 multiply-add
// finishes the index.
__device__ __forceinline__ int64_t cell_index(int w0, int w1, int w2, int n) {
  const uint32_t plane = uint32_t(w1) + __umul24(uint32_t(n), uint32_t(w2));
  return int64_t(uint64_t(uint32_t(w0)) + uint64_t(uint32_t(n)) * uint64_t(plane));
}

// one step of a wrapped coordinate
__device__ __forceinline__ int wrap_step(int w, int step, int n) {
  w += step;
  if (w >= n) w -= n;
  if (w < 0) w += n;
  return w;
}

// parametric distance from the source to the next plane of one axis: one
// division whatever the sign (lanes of a wavefront differ in it), +inf for a
// zero component
__device__ __forceinline__ double plane_t(double o, double d, int i) {
  const double t = (double(d > 0.0 ? i + 1 : i) - o) / d;
  return d != 0.0 ? t : __builtin_inf();
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

// The march's argument block, read through a pointer that the compiler must
// treat as new at every use: values read this way are re-read from the
// (scalar-cached) argument segment where they are used instead of being held
// in scalar registers across the whole loop.  The ray set-up reads its many
// pointers like this, which leaves the per-step path its registers.
using ArgsK = const MarchArgs __attribute__((address_space(4)));
__device__ __forceinline__ ArgsK& fresh_args() {
  ArgsK* p = (ArgsK*)__builtin_amdgcn_kernarg_segment_ptr();
  asm volatile("" : "+s"(p));
  return *p;
}

struct LaneAcc {
  double absorbed = 0.0, escaped = 0.0, truncated = 0.0;
  unsigned long long segments = 0;
};

// Per-wavefront Gamma accumulator in LDS.  A wavefront marches rays claimed
// in runs of consecutive queue entries; nested HEALPix order is a Z-order
// curve and children are queued next to each other, so such a run is a
// bundle of neighbouring pixels of one source and level, and by the split
// rule it crosses each cell several times.  Deposits are summed in an
// open-addressing hash table whose slots are 64-byte lines of Gamma (kLine
// consecutive cells along x), and folded into Gamma when a quarter of the
// slots are taken: the device performs FP64 atomics per 64-byte line
// request, so the flush, in which lanes 8j..8j+7 of an instruction cover the
// cells of one line, costs one request per line instead of one per cell.  A deposit that
// finds no slot within kProbe probes goes straight to Gamma.
constexpr int kWaves = kBlock / 64;
constexpr int kLine = 8;
constexpr int kProbe = 16;
constexpr uint32_t kEmpty = 0xffffffffu;

template <typename V>
struct LineTable {
  // line slots per wavefront: 36 KiB (FP32 sums) or 34 KiB (FP64) per block
  static constexpr int kLog2Lines = sizeof(V) == 4 ? 8 : 7;
  static constexpr int kLines = 1 << kLog2Lines;
  // fold at a quarter full: probe collisions cost more than the folds saved
  // (measured on the 1024^3 field: 1/4 84.3, 1/2 80.3, 3/4 68.8 G segments/s)
  static constexpr int kFlushAt = kLines / 4;
  static constexpr size_t kWaveBytes = kLines * (sizeof(uint32_t) + kLine * sizeof(V));

  uint32_t* key;  // [kLines] line index (cell >> 3) or kEmpty
  V* val;         // [kLines * kLine] partial sums of the line's cells
  bool on;        // false when line indices do not fit 32 bits below kEmpty

  // First probe for the line of cell c, issued ahead of the arithmetic that
  // precedes the deposit, so that the compare-and-swap is in flight while it
  // runs; `deposit` consumes its result.
  struct Claim {
    uint32_t k, h, old;
  };
  __device__ __forceinline__ Claim claim(int64_t c) const {
    Claim cl{uint32_t(c >> 3), 0u, 0u};
    if (on) {
      cl.h = (cl.k * 2654435761u) >> (32 - kLog2Lines);
      cl.old = atomicCAS(&key[cl.h], kEmpty, cl.k);
    }
    return cl;
  }
  // whether the claim took a new slot (it stays taken even if no value follows)
  __device__ __forceinline__ static bool took(const Claim& cl) { return cl.old == kEmpty; }

  // add v for cell c to the slot of its claim, probing further if the first
  // slot belongs to another line
  __device__ __forceinline__ int deposit(const Claim& cl, int64_t c, V v) const {
    if (on) {
      const uint32_t sub = uint32_t(c) & uint32_t(kLine - 1);
      if (cl.old == kEmpty || cl.old == cl.k) {
        atomicAdd(&val[cl.h * kLine + sub], v);
        return 0;
      }
      uint32_t h = cl.h;
#pragma unroll 1
      for (int probe = 1; probe < kProbe; ++probe) {
        h = (h + 1) & uint32_t(kLines - 1);
        const uint32_t old = atomicCAS(&key[h], kEmpty, cl.k);
        if (old == kEmpty || old == cl.k) {
          atomicAdd(&val[h * kLine + sub], v);
          return old == kEmpty ? 1 : 0;
        }
      }
    }
    atomicAdd(fresh_args().gamma + c, double(v));
    return 0;
  }

  // whole wavefront: fold the table into Gamma and clear it (LDS operations
  // of one wavefront complete in program order).  Cells of a line that got
  // no deposit hold zero and are skipped, so no address past the grid is
  // formed.
  __device__ __forceinline__ void flush(int lane) const {
    double* gamma = fresh_args().gamma;
    __builtin_amdgcn_wave_barrier();
    const int sub = lane & (kLine - 1);
    for (int q = lane / kLine; q < kLines; q += 64 / kLine) {
      const uint32_t k = key[q];
      if (k != kEmpty) {
        const V v = val[q * kLine + sub];
        if (v != V(0)) {
          atomicAdd(gamma + ((int64_t(k) << 3) + sub), double(v));
          val[q * kLine + sub] = V(0);
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
    for (int q = lane; q < kLines; q += 64) key[q] = kEmpty;
    __builtin_amdgcn_wave_barrier();
  }
};

// outcome of a step: keep marching, escaped, truncated, or split
constexpr int kGoOn = 0, kEscaped = 1, kTruncated = 2, kSplit = 3;
// cells a busy lane marches per iteration of the wavefront loop (measured on
// the 128^3, 512^3 and 1024^3 workloads: 1 -> 3 gains 4-5 %, 3 -> 4 about
// 1 %, 4 -> 8 another 0.5-3 %; the polychromatic march 1 -> 8 gains 5-11 %);
// a cell takes at most 2 new table slots, so a lane's count per iteration
// fits 5 bits
constexpr int kCellsPerIteration = 8;

// State of the ray a lane is marching.  Unwrapped cell coordinates (i) keep
// the plane crossings exact across periodic wraps; wrapped ones (w) address
// memory.
struct RayState {
  double o0, o1, o2, d0, d1, d2;
  double t0, t1, t2;
  double s, L;
  double tau;       // optical depth at the threshold (FP64, both paths)
  double P;         // photons carried (FP64 path)
  double T;         // mixed path: transmitted fraction
  float s_rate;     // mixed path: L / h^3 in FP32
  double a64;       // absorber of the current cell, loaded ahead
  int i0, i1, i2, w0, w1, w2;
  int level;
  uint32_t src, pix;
};

// ---- polychromatic sources: Phi(tau) = -ln F(tau) from the table ----
struct SpecPos {
  int q;         // interval
  double x;      // local coordinate in [0, 1)
  double inv_w;  // 1 / interval width in tau (a power of two)
};

// interval and local coordinate of tau >= 0, exactly, from the bits of 1 + tau
__device__ __forceinline__ SpecPos spec_pos(double tau) {
  constexpr int kShift = 52 - kSpecLog2Sub;
  const double v = 1.0 + tau;
  const uint64_t b = uint64_t(__double_as_longlong(v));
  const int e = int(b >> 52) - 1023;
  SpecPos p;
  p.q = (e << kSpecLog2Sub) + int((b >> kShift) & uint64_t(kSpecSub - 1));
  p.inv_w = __longlong_as_double((long long)(1023 + kSpecLog2Sub - e) << 52);
  p.x = (v - __longlong_as_double((long long)(b & ~((uint64_t(1) << kShift) - 1)))) * p.inv_w;
  return p;
}

// (p(x2) - p(x1)) / (x2 - x1) for p = c0 + c1 x + ... + c5 x^5, given
// c[0..4] = c1..c5, as sum_k c_k h_{k-1}(x1, x2) with h_j the complete
// homogeneous polynomial of degree j; free of cancellation, and p'(x1) when
// x2 = x1
template <typename T>
__device__ __forceinline__ T spec_slope(const T* c, T x1, T x2) {
  const T h1 = x1 + x2;
  const T x1s = x1 * x1;
  const T h2 = fma(x2, h1, x1s);
  const T x1c = x1s * x1;
  const T h3 = fma(x2, h2, x1c);
  const T h4 = fma(x2, h3, x1c * x1);
  return fma(c[4], h4, fma(c[3], h3, fma(c[2], h2, fma(c[1], h1, c[0]))));
}

// c1..c5 of interval q in the path's precision
template <bool MIXED, typename Args, typename V>
__device__ __forceinline__ void spec_coef(Args& A, int q, V* c) {
  if constexpr (MIXED) {
    const float4 lo = *reinterpret_cast<const float4*>(A.spec32[q].c);
    c[0] = lo.x;
    c[1] = lo.y;
    c[2] = lo.z;
    c[3] = lo.w;
    c[4] = A.spec32[q].c[4];
  } else {
    const double2* r = reinterpret_cast<const double2*>(A.spec64[q].c);
    const double2 a = r[0], b = r[1];
    c[0] = a.x;
    c[1] = a.y;
    c[2] = b.x;
    c[3] = b.y;
    c[4] = A.spec64[q].c[4];
  }
}

template <bool MIXED, typename Args>
__device__ __forceinline__ double spec_c0(Args& A, int q) {
  return MIXED ? A.spec32[q].c0 : A.spec64[q].c[5];
}

// Phi(tau) in FP64 (ray set-up); +inf past the table
template <typename Args>
__device__ double spec_phi(Args& A, double tau) {
  const SpecPos p = spec_pos(tau);
  if (p.q >= A.spec_nint) return __builtin_inf();
  double c[5];
  spec_coef<false>(A, p.q, c);
  return A.spec64[p.q].c[5] + p.x * spec_slope(c, 0.0, p.x);
}

// Rise of Phi over [tau, tau + dtau]: the optical depth that attenuates the
// whole spectrum across the cell, so that the cell absorbs the share
// 1 - e^{-rise} of the photons the ray carries.  `slope` receives the mean
// dPhi/dtau over the cell when the cell lies within one interval, which is
// dPhi/dtau at tau when dtau = 0 (the thin-cell limit).  Past the table's end
// the rise is infinite: the cell absorbs everything the ray still carries.
template <bool MIXED, typename Args, typename V>
__device__ __forceinline__ V spec_rise(Args& A, double tau, V dtau, V& slope) {
  const SpecPos p1 = spec_pos(tau);
  const SpecPos p2 = spec_pos(tau + double(dtau));
  V c[5];
  spec_coef<MIXED>(A, p1.q, c);
  if (p2.q == p1.q) {
    const V sl = spec_slope(c, V(p1.x), V(p2.x));
    slope = sl * V(p1.inv_w);
    return (dtau * V(p1.inv_w)) * sl;
  }
  slope = V(0);
  if (p2.q >= A.spec_nint) return V(__builtin_inf());
  // rest of the first interval, whole intervals between, start of the last
  const V first = (V(1) - V(p1.x)) * spec_slope(c, V(p1.x), V(1));
  spec_coef<MIXED>(A, p2.q, c);
  const V last = V(p2.x) * spec_slope(c, V(0), V(p2.x));
  const double mid = spec_c0<MIXED>(A, p2.q) - spec_c0<MIXED>(A, p1.q + 1);
  return (first + last) + V(mid);
}

// One ray of a launch as queued: source, HEALPix pixel, path length and
// optical depth at the threshold.  For injected rays `src` holds the ray's
// index.
struct Entry {
  uint32_t src, pix;
  double s, w;
};

// Entry r of the launch: a virtual spawn index, a queue slot or an injected
// ray's index.
template <typename Args>
__device__ __forceinline__ Entry load_entry(Args& A, int64_t r) {
  Entry e;
  if (A.level < 0) {
    e.src = uint32_t(r);
    e.pix = 0;
    e.s = 0.0;
    e.w = 0.0;
  } else if (A.spawn) {
    if (r < (int64_t(1) << 32)) {
      const uint32_t r32 = uint32_t(r);
      e.src = uint32_t(A.src_begin) + r32 / 12u;
      e.pix = r32 % 12u;
    } else {
      e.src = uint32_t(A.src_begin + r / 12);
      e.pix = uint32_t(r % 12);
    }
    e.s = 0.0;
    e.w = 0.0;
  } else {
    e.src = A.in.src[r];
    e.pix = A.in.pix[r];
    e.s = A.in.s[r];
    e.w = A.in.w[r];
  }
  return e;
}

// Start the ray of entry e: direction, start cell and first absorber.
// Returns kEscaped if it starts outside an open box, else kGoOn.
template <bool MIXED, bool PERIODIC, bool POLY, typename Args>
__device__ int ray_init(RayState& R, Args& A, const Entry& e) {
  double w = e.w;
  if (A.level < 0) {  // injected rays: never split
    const int64_t r = e.src;
    R.o0 = A.inj_origin[3 * r];
    R.o1 = A.inj_origin[3 * r + 1];
    R.o2 = A.inj_origin[3 * r + 2];
    R.d0 = A.inj_dir[3 * r];
    R.d1 = A.inj_dir[3 * r + 1];
    R.d2 = A.inj_dir[3 * r + 2];
    R.L = A.inj_L[r];
    R.level = A.inj_level[r];
    R.s = 0.0;
    R.src = R.pix = 0;
  } else {
    R.src = e.src;
    R.pix = e.pix;
    R.s = e.s;
    R.level = A.level;
    R.o0 = A.src_pos[3 * int64_t(R.src)];
    R.o1 = A.src_pos[3 * int64_t(R.src) + 1];
    R.o2 = A.src_pos[3 * int64_t(R.src) + 2];
    R.L = ldexp(A.src_l0[R.src], -2 * R.level);
    if (R.level <= A.dir_max_level) {  // the table holds this device function's values
      const double* d = A.dirs + 3 * (dir_table_offset(R.level) + int64_t(R.pix));
      R.d0 = d[0];
      R.d1 = d[1];
      R.d2 = d[2];
    } else {
      healpix_dir(R.level, R.pix, R.d0, R.d1, R.d2);
    }
  }
  R.i0 = start_cell(R.o0, R.s, R.d0);
  R.i1 = start_cell(R.o1, R.s, R.d1);
  R.i2 = start_cell(R.o2, R.s, R.d2);
  R.t0 = plane_t(R.o0, R.d0, R.i0);
  R.t1 = plane_t(R.o1, R.d1, R.i1);
  R.t2 = plane_t(R.o2, R.d2, R.i2);
  R.tau = w;
  // transmitted share of the ray's photons: e^{-tau}, or e^{-Phi(tau)} for a
  // spectrum (exactly 1 at a source)
  const double T = w == 0.0 ? 1.0 : exp(POLY ? -spec_phi(A, w) : -w);
  if (MIXED) {
    R.T = T;
    R.s_rate = float(R.L * A.inv_h3);
  } else {
    R.P = R.L * T;
  }
  const int n = A.n;
  const bool out = R.i0 < 0 || R.i0 >= n || R.i1 < 0 || R.i1 >= n || R.i2 < 0 || R.i2 >= n;
  if (!PERIODIC && out) return kEscaped;
  R.w0 = PERIODIC ? wrap_cell(R.i0, n) : R.i0;
  R.w1 = PERIODIC ? wrap_cell(R.i1, n) : R.i1;
  R.w2 = PERIODIC ? wrap_cell(R.i2, n) : R.i2;
  R.a64 = A.a64[cell_index(R.w0, R.w1, R.w2, n)];
  return kGoOn;
}


// Arguments every step reads, held in scalar registers for the whole
// launch.  Read from the argument block where they are used, the compiler
// would reload them there (scalar registers are scarce in the march), and the
// wait for such a load also waits for every LDS operation in flight.  An
// empty asm statement makes each value the output of an instruction, which
// cannot be reloaded, so it stays in a register.
struct StepConst {
  double s_max, tau_stop, sigma0;
  __device__ explicit StepConst(const MarchArgs& A)
      : s_max(A.s_max), tau_stop(A.tau_stop), sigma0(A.sigma0) {
    asm volatile("" : "+s"(s_max));
    asm volatile("" : "+s"(tau_stop));
    asm volatile("" : "+s"(sigma0));
  }
};

// Stop tests at the current cell boundary, then one cell segment: optical
// depth, Eq. lut_eqn deposit with the overlap correction, advance.  The
// caller books the photons of a ray that stops.  `inserted` counts new table
// slots taken by this call's deposits.  Memory latency is hidden by order:
// the cell's absorber was loaded at the end of the previous step; the
// neighbour's is requested by every lane (its own cell's when it needs no
// neighbour), so that the wait for the cell's word leaves that request in
// flight; the table claims are issued after the attenuation and before the
// advance, whose arithmetic covers them and the neighbour's load, and the
// deposits come last.
template <bool MIXED, int CORR, bool PERIODIC, bool POLY, typename V>
__device__ int ray_step(RayState& R, const MarchArgs& A, const LineTable<V>& tab, LaneAcc& acc,
                        int& inserted, const StepConst& K) {
  const int n = A.n;
  constexpr bool open_box = !PERIODIC;
  if (PERIODIC && R.s >= K.s_max) return kEscaped;
  // the optical-depth cap (for a spectrum: the threshold optical depth at
  // which the share of photons left falls to e^{-tau_max})
  if (R.tau >= K.tau_stop) return kTruncated;
  // split radius^2 of the launch's level (injected rays never split)
  const double r2s = A.level < 0 ? __builtin_inf() : A.r2split;
  if (R.s * R.s > r2s) return R.level >= A.l_max ? kTruncated : kSplit;
  // next crossing: lowest axis wins exact ties
  int ax = 0;
  double tn = R.t0;
  if (R.t1 < tn) {
    ax = 1;
    tn = R.t1;
  }
  if (R.t2 < tn) {
    ax = 2;
    tn = R.t2;
  }
  double ds = tn - R.s;
  if (ds < 0.0) ds = 0.0;
  const int64_t c = cell_index(R.w0, R.w1, R.w2, n);

  // ---- overlap geometry (Eqs. correction .. new_secondary): nearest face
  // of the segment midpoint, and the neighbour across it ----
  bool near = false;
  double dedge = 0.0, lpix = 1.0;
  bool neighbour = false;  // the neighbour's absorber is needed
  int64_t c2 = 0;
  double raw2_64 = 0.0;
  float raw2_32 = 0.0f;
  if constexpr (CORR != NRT_CORR_NONE) {
    const double rm = 0.5 * (R.s + tn);
    // sqrt of the pixel solid angle: sqrt(Omega(0)) 2^-level, exactly
    lpix = rm * ldexp(A.sqrt_omega_tab[0], -R.level);
    // per axis: distance to the nearer face and its side (-1 lower, +1
    // upper; an exact tie goes the way the ray points); the first axis wins
    // ties between axes.  Selects only, no branches.
    const double m0 = R.o0 + rm * R.d0;
    const double dm0 = m0 - double(R.i0), dp0 = double(R.i0 + 1) - m0;
    const double m1 = R.o1 + rm * R.d1;
    const double dm1 = m1 - double(R.i1), dp1 = double(R.i1 + 1) - m1;
    const double m2 = R.o2 + rm * R.d2;
    const double dm2 = m2 - double(R.i2), dp2 = double(R.i2 + 1) - m2;
    // both comparisons up front, so that the side is two selects
    const bool lt0 = dm0 < dp0, gt0 = dp0 < dm0;
    const bool lt1 = dm1 < dp1, gt1 = dp1 < dm1;
    const bool lt2 = dm2 < dp2, gt2 = dp2 < dm2;
    const int s0 = lt0 ? -1 : (gt0 ? 1 : (R.d0 < 0.0 ? -1 : 1));
    const int s1 = lt1 ? -1 : (gt1 ? 1 : (R.d1 < 0.0 ? -1 : 1));
    const int s2 = lt2 ? -1 : (gt2 ? 1 : (R.d2 < 0.0 ? -1 : 1));
    const double da0 = lt0 ? dm0 : dp0;
    const double da1 = lt1 ? dm1 : dp1;
    const double da2 = lt2 ? dm2 : dp2;
    const bool b1 = da1 < da0;
    const double d01 = b1 ? da1 : da0;
    const bool b2 = da2 < d01;
    dedge = b2 ? da2 : d01;
    const int fax = b2 ? 2 : (b1 ? 1 : 0);
    const int fdir = b2 ? s2 : (b1 ? s1 : s0);
    near = dedge < 0.5 * lpix;
    if (near && (CORR == NRT_CORR_CONSERVATIVE || CORR == NRT_CORR_NAIVE)) {
      // the neighbour differs from the cell in the face's axis only
      const int i_f = fax == 0 ? R.i0 : (fax == 1 ? R.i1 : R.i2);
      const int j_f = i_f + fdir;
      if (!open_box || !(j_f < 0 || j_f >= n)) {
        const int w_f = open_box ? i_f : (fax == 0 ? R.w0 : (fax == 1 ? R.w1 : R.w2));
        const int v_f = open_box ? j_f : wrap_step(w_f, fdir, n);
        // n^2 <= 2^24 fits 32 bits: one 32 x 32 -> 64 signed multiply
        const int32_t stride = fax == 0 ? 1 : (fax == 1 ? n : n * n);
        c2 = c + int64_t(v_f - w_f) * int64_t(stride);
        neighbour = true;
      }
    }
    // requested by every lane, whether or not it needs a neighbour, so the
    // load is never skipped by a branch and the wait for this cell's word
    // below can leave it in flight
    if constexpr (CORR == NRT_CORR_CONSERVATIVE || CORR == NRT_CORR_NAIVE)
      raw2_64 = A.a64[neighbour ? c2 : c];
  }

  // ---- segment physics (Eq. lut_eqn, Eq. optical_depth) ----
  // the cell's optical depth in FP64, the same operations in both paths
  const double a64 = fabs(R.a64);
  const double dl = ds * A.h_cm;
  const double dtau64 = K.sigma0 * a64 * dl;
  double G64 = 0.0;
  float G32 = 0.0f, a32 = 0.0f;
  if (MIXED) {
    a32 = float(a64);
    const float dsf = float(ds);
    float dtau = float(dtau64);
    float slope32 = 1.0f;
    if constexpr (POLY) {  // the whole spectrum's attenuation across the cell
      const float dtau0 = dtau;
      dtau = spec_rise<true>(A, R.tau, dtau0, slope32);
    }
    R.tau += dtau64;
    // surviving share e = exp(-dtau) from the hardware base-2 exponential
    // (1 ulp); absorbed share em = 1 - e, which for dtau < 1/8 comes from
    // its series (relative truncation error below dtau^5/720 < 5e-8) since
    // 1 - e would cancel there
    const float e = __builtin_amdgcn_exp2f(dtau * -1.44269504f);
    const float poly =
        dtau * fmaf(dtau, fmaf(dtau, fmaf(dtau, fmaf(dtau, 1.0f / 120.0f, -1.0f / 24.0f),
                                          1.0f / 6.0f), -0.5f), 1.0f);
    const float em = dtau < 0.125f ? poly : 1.0f - e;
    // transmitted fraction in FP64: the absorbed part for weak absorption,
    // the surviving part for strong absorption (where em rounds towards 1)
    double dT, Tn;
    if (em < 0.5f) {
      dT = R.T * double(em);
      Tn = R.T - dT;
    } else {
      Tn = R.T * double(e);
      dT = R.T - Tn;
    }
    const float Tf = float(R.T);
    R.T = Tn;
    acc.absorbed = fma(R.L, dT, acc.absorbed);
    // an absorber below FP32's normal range takes the thin limit, which is
    // exact there
    G32 = a32 >= FLT_MIN ? (R.s_rate * float(dT)) * __builtin_amdgcn_rcpf(a32)
                         : R.s_rate * Tf * (A.kf * dsf) * slope32;
  } else {
    double rise = dtau64, slope64 = 1.0;
    if constexpr (POLY) rise = spec_rise<false>(A, R.tau, dtau64, slope64);
    const double dN = R.P * (-expm1(-rise));
    G64 = a64 > 0.0 ? dN / (a64 * A.h3) : R.P * A.sigma0 * dl * slope64 / A.h3;
    acc.absorbed += dN;
    R.P -= dN;
    R.tau += dtau64;
  }

  // ---- table claims, in flight during the advance ----
  const auto cl1 = tab.claim(c);
  typename LineTable<V>::Claim cl2{0u, 0u, 0u};
  if (neighbour) cl2 = tab.claim(c2);

  // ---- advance one cell: step the winning axis (its component is nonzero)
  // and recompute its next plane crossing, without diverging on the axis ----
  R.s = tn;
  {
    // the winning axis's fields by two selects each (32-bit selects, cheaper
    // than masked FP64 sums)
    const bool a0 = ax == 0, a1 = ax == 1;
    const double o_a = a0 ? R.o0 : (a1 ? R.o1 : R.o2);
    const double d_a = a0 ? R.d0 : (a1 ? R.d1 : R.d2);
    const int st_a = d_a > 0.0 ? 1 : -1;
    const int i_a = (a0 ? R.i0 : (a1 ? R.i1 : R.i2)) + st_a;
    const int w_a = open_box ? i_a : wrap_step(a0 ? R.w0 : (a1 ? R.w1 : R.w2), st_a, n);
    const double t_a = (double(st_a > 0 ? i_a + 1 : i_a) - o_a) / d_a;
    R.i0 = ax == 0 ? i_a : R.i0;
    R.i1 = ax == 1 ? i_a : R.i1;
    R.i2 = ax == 2 ? i_a : R.i2;
    R.w0 = ax == 0 ? w_a : R.w0;
    R.w1 = ax == 1 ? w_a : R.w1;
    R.w2 = ax == 2 ? w_a : R.w2;
    R.t0 = ax == 0 ? t_a : R.t0;
    R.t1 = ax == 1 ? t_a : R.t1;
    R.t2 = ax == 2 ? t_a : R.t2;
  }
  acc.segments += 1;
  const bool escaped = open_box &&
      (R.i0 < 0 || R.i0 >= n || R.i1 < 0 || R.i1 >= n || R.i2 < 0 || R.i2 >= n);
  // absorber of the next cell, consumed by the next step (a ray that left
  // the open box reads its last cell's instead)
  R.a64 = A.a64[escaped ? c : cell_index(R.w0, R.w1, R.w2, n)];

  // ---- overlap correction values (the decision above is FP64; the factor
  // is FP32 in the mixed path) ----
  using R_t = typename std::conditional<MIXED, float, double>::type;
  R_t fc = R_t(1);
  bool secondary = false;
  if (near) {
    const bool usable = neighbour && !__builtin_signbit(raw2_64);
    // the mixed path's FP32 neighbour absorber, floored at the smallest
    // normal so that its reciprocal stays finite
    if (MIXED) raw2_32 = fmaxf(float(raw2_64), FLT_MIN);
    R_t f;
    if constexpr (MIXED)
      f = 0.5f + float(dedge) * __builtin_amdgcn_rcpf(float(lpix));
    else
      f = 0.5 + dedge / lpix;
    if constexpr (CORR == NRT_CORR_LINEAR) {
      fc = f;
    } else if constexpr (CORR == NRT_CORR_SQUARED) {
      fc = f * f;
    } else if constexpr (CORR == NRT_CORR_CONSERVATIVE) {
      if (usable) fc = f;
      secondary = usable;
    } else {  // NAIVE
      fc = f;
      secondary = usable;
    }
  }

  // ---- deposit ----
  inserted += LineTable<V>::took(cl1) ? 1 : 0;
  if (neighbour) inserted += LineTable<V>::took(cl2) ? 1 : 0;
  if constexpr (MIXED) {
    inserted += tab.deposit(cl1, c, fc * G32);
    if (secondary)
      inserted += tab.deposit(cl2, c2, ((1.0f - fc) * (a32 * __builtin_amdgcn_rcpf(raw2_32))) * G32);
  } else {
    inserted += tab.deposit(cl1, c, fc * G64);
    if (secondary) inserted += tab.deposit(cl2, c2, ((1.0 - fc) * (a64 / raw2_64)) * G64);
  }

  return escaped ? kEscaped : kGoOn;
}

// Whole wavefront: append the four children of every lane with a pending
// split to the next level's queue (one atomicAdd for the wavefront).
__device__ __forceinline__ void push_pending(unsigned long long* count, const RayQueue& out,
                                             int64_t out_cap, unsigned long long* overflow,
                                             int lane, bool& pend, uint32_t p_src,
                                             uint32_t p_pix, double p_s, double p_w) {
  const uint64_t pm = __ballot(pend);
  if (!pm) return;
  const int leader = __builtin_ctzll(pm);
  unsigned long long slot0 = 0;
  if (lane == leader) slot0 = atomicAdd(count, 4ull * static_cast<unsigned long long>(__popcll(pm)));
  slot0 = read_lane64(slot0, leader);
  if (pend) {
    const unsigned long long slot = slot0 + 4ull * lanes_below(pm);
    if (slot + 4 <= static_cast<unsigned long long>(out_cap)) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        out.src[slot + k] = p_src;
        out.pix[slot + k] = 4u * p_pix + uint32_t(k);
        out.s[slot + k] = p_s;
        out.w[slot + k] = p_w;
      }
    } else {
      atomicAdd(overflow, 1ull);
    }
    pend = false;
  }
}

// Persistent march: every wavefront takes runs of A.claim rays of the
// launch's range (its first by position, the rest from a shared counter),
// refills idle lanes from its run once A.refill_min of them are idle,
// advances every busy lane by up to 8 cells per iteration, and folds its
// LDS table into Gamma when a quarter full.  A lane whose ray splits keeps the
// children's start state in registers; the wavefront appends the children of
// all pending splits to the next level's queue with one atomicAdd once every
// lane holds one (or a pending lane splits again, or the wavefront is done):
// fewer same-address atomics than a push at 32 (1024^3: +1.3 % mixed, +4 %
// FP64).
// The mixed march is held to 128 VGPRs, which keeps 4 waves per SIMD as its
// LDS allows (it fits with no VGPR spills), except the open-box
// polychromatic one, which would spill under that cap; it and the FP64
// march are left to the compiler (3 waves per SIMD).
template <bool MIXED, int CORR, bool PERIODIC, bool POLY>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu((MIXED && (PERIODIC || !POLY)) ? 4 : 1, 8))) void k_march(
    MarchArgs A) {
  if (A.skip && *A.skip) return;  // a replayed pass after its iteration stopped
  using V = typename std::conditional<MIXED, float, double>::type;
  // per-wavefront deposit tables, reused for the budget reduction at the end
  using Tab = LineTable<V>;
  __shared__ __align__(16) unsigned char lds[kWaves * Tab::kWaveBytes];
  const int wave = threadIdx.x >> 6;
  const int lane = __lane_id();
  uint32_t* key = reinterpret_cast<uint32_t*>(lds) + wave * Tab::kLines;
  V* val = reinterpret_cast<V*>(lds + kWaves * Tab::kLines * sizeof(uint32_t)) +
           wave * Tab::kLines * kLine;
  const Tab tab{key, val, A.lds_keys_fit != 0};
  for (int q = lane; q < Tab::kLines; q += 64) key[q] = kEmpty;
  for (int q = lane; q < Tab::kLines * kLine; q += 64) val[q] = V(0);
  __builtin_amdgcn_wave_barrier();

  LaneAcc acc;
  RayState R;
  bool busy = false;
  // pending split of this lane: children start state
  bool pend = false;
  uint32_t p_src = 0, p_pix = 0;
  double p_s = 0.0, p_w = 0.0;
  int64_t total = A.end - A.begin;
  if (A.count_src) {
    const int64_t k = int64_t(*A.count_src);
    total = k < A.in_cap ? k : A.in_cap;
  }
  // Wavefront w starts with rays [w claim, (w+1) claim) of the launch's range
  // without touching the shared counter, which hands out the runs after the
  // first nwaves * claim.  A wavefront with no first run has nothing to do,
  // so the idle part of a persistent grid (small levels) issues no atomics.
  const int64_t claim = A.claim;
  const int64_t first_runs = int64_t(gridDim.x) * kWaves * claim;
  // the run bounds are wavefront-uniform: derive them from a uniform wave
  // index so that they stay in scalar registers
  const int wave_u = __builtin_amdgcn_readfirstlane(wave);
  int64_t pool = (int64_t(blockIdx.x) * kWaves + wave_u) * claim;
  int64_t pool_end = pool + claim < total ? pool + claim : total;
  bool exhausted = pool >= total;
  if (exhausted) pool = pool_end = 0;
  const StepConst K(A);
  int fill = 0;                    // wavefront-uniform occupied line slots
  for (;;) {
    const uint64_t idle = __ballot(!busy);
    const int n_idle = __popcll(idle);
    if (!exhausted && (n_idle >= A.refill_min || n_idle == 64)) {
      ArgsK& F = fresh_args();
      if (pool == pool_end) {
        unsigned long long b = 0;
        if (lane == 0) b = atomicAdd(F.claim_ctr, static_cast<unsigned long long>(claim));
        b = read_lane64(b, 0) + static_cast<unsigned long long>(first_runs);
        if (int64_t(b) >= total) {
          exhausted = true;
        } else {
          pool = int64_t(b);
          pool_end = int64_t(b) + claim < total ? int64_t(b) + claim : total;
        }
      }
      if (!exhausted) {
        const int64_t avail = pool_end - pool;
        const unsigned rank = lanes_below(idle);
        if (!busy && int64_t(rank) < avail) {
          const Entry e = load_entry(F, F.begin + pool + rank);
          const int start = ray_init<MIXED, PERIODIC, POLY>(R, F, e);
          busy = start == kGoOn;
          if (!busy) acc.escaped += MIXED ? R.L * R.T : R.P;
        }
        pool += int64_t(n_idle) < avail ? int64_t(n_idle) : avail;
      }
    }
    if (__ballot(busy) == 0) {
      if (exhausted) break;
      continue;
    }
    // a few cells per busy lane between the wavefront's bookkeeping (refill,
    // split pushes, table occupancy); a lane that stops sits out the rest
    int code = kGoOn, inserted = 0;
#pragma unroll 1
    for (int k = 0; k < kCellsPerIteration && busy; ++k) {
      code = ray_step<MIXED, CORR, PERIODIC, POLY>(R, A, tab, acc, inserted, K);
      if (code != kGoOn) {
        busy = false;
        const double carried = MIXED ? R.L * R.T : R.P;
        acc.escaped += code == kEscaped ? carried : 0.0;
        acc.truncated += code == kTruncated ? carried : 0.0;
      }
    }
    fill += __popcll(__ballot(inserted & 1)) + 2 * __popcll(__ballot(inserted & 2)) +
            4 * __popcll(__ballot(inserted & 4)) + 8 * __popcll(__ballot(inserted & 8)) +
            16 * __popcll(__ballot(inserted & 16));
    const bool splits = code == kSplit;
    if (__ballot(splits && pend)) {  // a lane splits again
      ArgsK& F = fresh_args();
      const RayQueue out{F.out.src, F.out.pix, F.out.s, F.out.w};
      push_pending(&F.acc->out_count[F.level + 1], out, F.out_cap, &F.acc->overflow, lane, pend,
                   p_src, p_pix, p_s, p_w);
    }
    if (splits) {
      pend = true;
      p_src = R.src;
      p_pix = R.pix;
      p_s = R.s;
      p_w = R.tau;
    }
    if (__ballot(pend) == ~0ull) {  // every lane holds a pending split
      ArgsK& F = fresh_args();
      const RayQueue out{F.out.src, F.out.pix, F.out.s, F.out.w};
      push_pending(&F.acc->out_count[F.level + 1], out, F.out_cap, &F.acc->overflow, lane, pend,
                   p_src, p_pix, p_s, p_w);
    }
    if (fill >= Tab::kFlushAt) {
      tab.flush(lane);
      fill = 0;
    }
  }
  push_pending(&A.acc->out_count[A.level + 1], A.out, A.out_cap, &A.acc->overflow, lane, pend,
               p_src, p_pix, p_s, p_w);
  tab.flush(lane);

  // block reduction of the lane budgets, then one atomic per block and term
  __syncthreads();
  static_assert(kWaves * Tab::kWaveBytes >= kBlock * 32, "reduction space");
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
  if (threadIdx.x == 0 && (red_u[0] != 0 || red_d[1][0] != 0.0 || red_d[2][0] != 0.0)) {
    // a block that marched nothing and stopped no ray adds nothing
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
                       int64_t ncell, double* a64, Accum* acc,
                       const unsigned long long* skip) {
  if (skip && *skip) return;
  unsigned long long bad = 0;
  for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < ncell;
       c += int64_t(gridDim.x) * blockDim.x) {
    const double nh = n_H[c], xx = x[c];
    if (!(nh >= 0.0) || isinf(nh) || !(xx >= 0.0 && xx <= 1.0)) ++bad;
    const double a = (1.0 - xx) * nh;
    const bool usable = nh >= n_th && a > 0.0;
    a64[c] = usable ? a : -a;
  }
  if (bad) atomicAdd(&acc->invalid, bad);
}

// The threshold optical depth at which a spectrum's Phi reaches tau_max:
// the smallest tau with Phi(tau) >= tau_max on the FP64 table, to the last
// bit, by bisection of [0, hi] (Phi(0) = 0 < tau_max and Phi(hi) >= tau_max
// at the table's end).  The march stops a ray once its threshold optical
// depth reaches it, which is the photon-share cap F <= e^{-tau_max} taken on
// an FP64 quantity that both precisions accumulate alike.  One thread.
struct SpecTable {
  int32_t spec_nint;
  const SpecRec64* spec64;
  const SpecRec32* spec32;
};

__global__ void k_spec_stop(SpecTable t, double tau_max, double hi, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double lo = 0.0;
  for (int it = 0; it < 4096; ++it) {
    const double mid = lo + 0.5 * (hi - lo);
    if (!(mid > lo && mid < hi)) break;
    if (spec_phi(t, mid) >= tau_max)
      hi = mid;
    else
      lo = mid;
  }
  *out = hi;
}

__global__ void k_fill_zero(double* p, int64_t count, const unsigned long long* skip) {
  if (skip && *skip) return;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = 0.0;
}

__global__ void k_zero_accum(Accum* acc, const unsigned long long* skip) {
  if (skip && *skip) return;
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

__global__ void k_budget(const Accum* acc, nrt_budget* out, uint64_t* dropped, double emitted,
                         uint64_t spawned, int l_max) {
  if (threadIdx.x != 0) return;
  nrt_budget b;
  b.emitted = emitted;
  b.absorbed = acc->absorbed;
  b.escaped = acc->escaped;
  b.truncated = acc->truncated;
  b.segments = acc->segments;
  b.rays = 0;
  b.splits = 0;
  for (int l = 0; l <= NRT_MAX_LEVEL; ++l) {
    const uint64_t k = l == 0 ? spawned : (l <= l_max ? uint64_t(acc->out_count[l]) : 0);
    b.rays_per_level[l] = k;
    b.rays += k;
    if (l > 0) b.splits += k / 4;
  }
  *out = b;
  if (dropped) *dropped = acc->overflow;
}

__global__ void k_rt_check(const Accum* acc, RtState* rt, unsigned long long threshold,
                           unsigned long long max_iter) {
  if (threadIdx.x != 0 || rt->done) return;
  rt->iters += 1;
  rt->changed = acc->chem_changed;
  rt->overflow |= acc->overflow;
  rt->invalid |= acc->invalid;
  if (rt->invalid || rt->overflow || acc->chem_changed <= threshold || rt->iters >= max_iter)
    rt->done = 1;
}

__global__ void k_rt_reset(RtState* rt) {
  unsigned long long* p = reinterpret_cast<unsigned long long*>(rt);
  for (int i = threadIdx.x; i < int(sizeof(RtState) / 8); i += blockDim.x) p[i] = 0ull;
}

int grid_for(int64_t items, int block, int cap) {
  int64_t g = (items + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return int(g);
}

}  // namespace

hipError_t launch_prep_fields(const double* n_H, const double* x, double n_th, int64_t ncell,
                              double* a64, Accum* acc, int cus, hipStream_t s) {
  hipLaunchKernelGGL(k_prep, dim3(grid_for(ncell, 256, cus * 16)), dim3(256), 0, s, n_H, x, n_th,
                     ncell, a64, acc, nullptr);
  return hipGetLastError();
}

hipError_t launch_prep_from(nrt_ctx* c, const double* x, const unsigned long long* skip,
                            hipStream_t s) {
  const int64_t ncell = c->lay.cells;
  hipLaunchKernelGGL(k_prep, dim3(grid_for(ncell, 256, c->cu_count * 16)), dim3(256), 0, s,
                     c->n_H, x, c->desc.n_th, ncell, c->a64, c->acc, skip);
  return hipGetLastError();
}

hipError_t launch_rt_check(const Accum* acc, RtState* rt, unsigned long long threshold,
                           unsigned long long max_iter, hipStream_t s) {
  hipLaunchKernelGGL(k_rt_check, dim3(1), dim3(64), 0, s, acc, rt, threshold, max_iter);
  return hipGetLastError();
}

hipError_t launch_rt_reset(RtState* rt, hipStream_t s) {
  hipLaunchKernelGGL(k_rt_reset, dim3(1), dim3(64), 0, s, rt);
  return hipGetLastError();
}

hipError_t launch_prep(nrt_ctx* c) {
  return launch_prep_fields(c->n_H, c->x, c->desc.n_th, c->lay.cells, c->a64, c->acc,
                            c->cu_count, c->stream);
}

hipError_t launch_spec_stop(const nrt_ctx* c, double* out) {
  const SpecTable t{c->spec_nint, c->spec64, c->spec32};
  // the table ends at an octave boundary: node tau 2^octaves - 1
  const double hi = std::ldexp(1.0, c->spec_nint >> kSpecLog2Sub) - 1.0;
  hipLaunchKernelGGL(k_spec_stop, dim3(1), dim3(64), 0, c->stream, t, c->desc.tau_max, hi, out);
  return hipGetLastError();
}

hipError_t launch_zero(double* p, int64_t count, int cus, hipStream_t s,
                       const unsigned long long* skip) {
  hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(count, 256, cus * 16)), dim3(256), 0, s, p,
                     count, skip);
  return hipGetLastError();
}

hipError_t launch_zero_accum(Accum* acc, hipStream_t s, const unsigned long long* skip) {
  hipLaunchKernelGGL(k_zero_accum, dim3(1), dim3(256), 0, s, acc, skip);
  return hipGetLastError();
}

namespace {

// the march instantiation for a precision, correction mode, boundary and spectrum
using MarchKernel = void (*)(MarchArgs);

template <bool MIXED, bool PERIODIC, bool POLY>
MarchKernel march_for_corr(int corr) {
  switch (corr) {
    case NRT_CORR_NONE: return k_march<MIXED, NRT_CORR_NONE, PERIODIC, POLY>;
    case NRT_CORR_LINEAR: return k_march<MIXED, NRT_CORR_LINEAR, PERIODIC, POLY>;
    case NRT_CORR_SQUARED: return k_march<MIXED, NRT_CORR_SQUARED, PERIODIC, POLY>;
    case NRT_CORR_NAIVE: return k_march<MIXED, NRT_CORR_NAIVE, PERIODIC, POLY>;
    default: return k_march<MIXED, NRT_CORR_CONSERVATIVE, PERIODIC, POLY>;
  }
}

template <bool POLY>
MarchKernel march_for_spectrum(const nrt_grid_desc& d) {
  if (d.precision == NRT_MIXED)
    return d.periodic ? march_for_corr<true, true, POLY>(d.corr)
                      : march_for_corr<true, false, POLY>(d.corr);
  return d.periodic ? march_for_corr<false, true, POLY>(d.corr)
                    : march_for_corr<false, false, POLY>(d.corr);
}

MarchKernel march_kernel(const nrt_grid_desc& d) {
  return d.spectrum != NRT_SPEC_MONO ? march_for_spectrum<true>(d)
                                     : march_for_spectrum<false>(d);
}

}  // namespace

hipError_t march_blocks_per_cu(const nrt_grid_desc& d, int* blocks) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, march_kernel(d), kBlock, 0);
}

// persistent grid: as many blocks as stay resident, or fewer for small launches
hipError_t launch_march_on(const nrt_grid_desc& d, int cu_count, int resident_per_cu,
                           const nrt_tuning& t, const MarchArgs& args, int64_t rays,
                           hipStream_t st) {
  int per_cu = resident_per_cu > 0 ? resident_per_cu : 2;
  if (t.blocks_per_cu > 0 && t.blocks_per_cu < per_cu) per_cu = t.blocks_per_cu;
  const int blocks = grid_for(rays, kBlock, cu_count * per_cu);
  MarchArgs a = args;
  // defaults from sweeps of the device-driven pass on the 128^3, 256^3 and
  // 512^3 workloads: runs of two wavefronts of rays halve the claims of
  // short-ray workloads without starving waves at the end of a level; a
  // refill once 16 lanes idle amortizes the ray set-up
  a.claim = t.claim > 0 ? t.claim : 128;
  a.refill_min = t.refill_min > 0 ? t.refill_min : 16;
  hipLaunchKernelGGL(march_kernel(d), dim3(blocks), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_march(const nrt_ctx* c, const MarchArgs& args, int64_t rays, hipStream_t st) {
  return launch_march_on(c->desc, c->cu_count, c->march_blocks_per_cu, c->tuning, args, rays,
                         st);
}

namespace {
// l0[k] = ndot[k] / 12, the rate of a level-0 ray (a correctly rounded
// division, as on the host)
__global__ void k_source_rates(const double* ndot, int64_t m, double* l0) {
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < m;
       k += int64_t(gridDim.x) * blockDim.x)
    l0[k] = ndot[k] / 12.0;
}
}  // namespace

hipError_t launch_source_rates(const double* ndot, int64_t m, double* l0, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_source_rates, dim3(grid_for(m, 256, 1024)), dim3(256), 0, s, ndot, m, l0);
  return hipGetLastError();
}

hipError_t launch_budget(const Accum* acc, nrt_budget* out, uint64_t* dropped, double emitted,
                         int64_t spawned, int l_max, hipStream_t s) {
  hipLaunchKernelGGL(k_budget, dim3(1), dim3(64), 0, s, acc, out, dropped, emitted,
                     uint64_t(spawned), l_max);
  return hipGetLastError();
}

hipError_t launch_healpix(int level, int64_t first, int64_t count, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_healpix, dim3(grid_for(count, 256, 1 << 20)), dim3(256), 0, s, level,
                     first, count, out);
  return hipGetLastError();
}

}  // namespace nrt
