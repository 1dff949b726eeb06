// Device side of libpmc: precision policy, Philox4x32-10, per-lane proton
// state and the condensed-history step shared by every transport kernel.
//
// One history per lane.  The step follows the class II scheme of the design
// notes: restricted-stopping continuous loss through the range table,
// Gaussian soft straggling, explicit hard delta rays absorbed locally,
// telescoping Highland scattering and nuclear removal, with the dose tallied
// as int64 fixed-point (2^-32 MeV) so that the result does not depend on the
// order of the atomic updates (the paper sums energy with atomics, Sec. 2.D.2).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pmc_internal.hpp"

namespace pmc {

// ---------------------------------------------------------------------------
// constants of the transport model
// ---------------------------------------------------------------------------
constexpr double kMe = 0.51099895;
constexpr double kMp = 938.27208816;
constexpr double kX0 = 36.08;
constexpr double kElo = 1.0;
constexpr double kEhi = 300.0;
constexpr double kTcut = 0.1;
constexpr double kMuN = 0.0115;
constexpr double kEn = 10.0;
constexpr double kEpsR = 0.1;
constexpr double kSfloor = 0.01;
constexpr int kNtab = 1024;
constexpr int kLutSize = 4096;  // integer HU -1024 .. 3071
constexpr int kHuMin = -1024;
constexpr int kHuMax = 3071;
constexpr uint32_t kMaxSteps = 1u << 20;

enum : uint32_t {
  kNoStraggling = 1u, kNoMcs = 2u, kNoDelta = 4u, kNoNuclear = 8u, kFrozen = 16u
};
enum : int { kStop = 0, kGeo = 1, kDelta = 2, kNuc = 3, kPhys = 4 };
enum : int { kAlive = 0, kStopped = 1, kEscaped = 2, kNuclear = 3, kMissed = 4 };

// counter block layout (uint64 words)
enum : int {
  kCEscLo = 0, kCEscHi, kCNucLo, kCNucHi, kCCutLo, kCCutHi,
  kCHist, kCSteps, kCDelta, kCNucEv, kCEscapes, kCMisses, kCAtomics, kCSpare0, kCSpare1, kCSpare2
};

// ---------------------------------------------------------------------------
// precision policy
// ---------------------------------------------------------------------------
template <typename R> struct M;

template <> struct M<float> {
  using R2 = float2;
  using R4 = float4;
  static __device__ __forceinline__ float log2(float x) { return __builtin_amdgcn_logf(x); }
  static __device__ __forceinline__ float exp2(float x) { return __builtin_amdgcn_exp2f(x); }
  static __device__ __forceinline__ float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
  static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
  static __device__ __forceinline__ float div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
  // cos / sin of 2 pi u for u in [0, 1): the hardware takes revolutions
  static __device__ __forceinline__ float cos_rev(float u) { return __builtin_amdgcn_cosf(u); }
  static __device__ __forceinline__ float sin_rev(float u) { return __builtin_amdgcn_sinf(u); }
  static __device__ __forceinline__ float uni(uint32_t x) {
    return ((float)(x >> 8) + 0.5f) * 0x1p-24f;
  }
  // fixed-point energy Q(E) = E * 2^32, exact for float E >= 2^-9: with
  // E = m 2^(e-23) (m the 24-bit significand) it is m << (e + 9).  Transport
  // only asks for E >= 1 MeV (or exactly 0).
  static __device__ __forceinline__ long long q(float E) {
    const uint32_t b = __float_as_uint(E);
    const int sh = (int)(b >> 23) - 127 + 9;
    const unsigned long long m = (unsigned long long)((b & 0x7FFFFFu) | 0x800000u);
    return E == 0.0f ? 0ll : (long long)(m << sh);
  }
  // 1 - 2^-y for y >= 0.  1 - exp2(-y) cancels for the small y of a step
  // through air (its absolute error is an ulp of 1); below z = y ln 2 = 1/16
  // the series z - z^2/2 + z^3/6 - z^4/24 is used, whose first omitted term
  // is under 2^-23 of the result.
  static __device__ __forceinline__ float one_minus_exp2_neg(float y) {
    const float z = y * 0.693147180559945309f;
    if (z < 0.0625f) return z * (1.0f - z * (0.5f - z * (1.0f / 6.0f - z * (1.0f / 24.0f))));
    return 1.0f - __builtin_amdgcn_exp2f(-y);
  }
  static __device__ __forceinline__ float inf() { return __builtin_huge_valf(); }
  static __device__ __forceinline__ float fmax(float a, float b) { return __builtin_fmaxf(a, b); }
  static __device__ __forceinline__ float fmin(float a, float b) { return __builtin_fminf(a, b); }
};

template <> struct M<double> {
  using R2 = double2;
  using R4 = double4;
  static __device__ __forceinline__ double log2(double x) { return ::log2(x); }
  static __device__ __forceinline__ double exp2(double x) { return ::exp2(x); }
  static __device__ __forceinline__ double sqrt(double x) { return ::sqrt(x); }
  static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
  static __device__ __forceinline__ double div(double a, double b) { return a / b; }
  static __device__ __forceinline__ double cos_rev(double u) {
    return ::cos(6.283185307179586476925286766559 * u);
  }
  static __device__ __forceinline__ double sin_rev(double u) {
    return ::sin(6.283185307179586476925286766559 * u);
  }
  static __device__ __forceinline__ double uni(uint32_t x) { return ((double)x + 0.5) * 0x1p-32; }
  static __device__ __forceinline__ long long q(double E) { return __double2ll_rn(E * 4294967296.0); }
  static __device__ __forceinline__ double one_minus_exp2_neg(double y) {
    return -::expm1(-y * 0.69314718055994530942);
  }
  static __device__ __forceinline__ double inf() { return __builtin_huge_val(); }
  static __device__ __forceinline__ double fmax(double a, double b) { return __builtin_fmax(a, b); }
  static __device__ __forceinline__ double fmin(double a, double b) { return __builtin_fmin(a, b); }
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // 32 x 32 -> 64-bit products: one multiply-add instruction each
    const unsigned long long p0 = (unsigned long long)c0 * 0xD2511F53u;
    const unsigned long long p1 = (unsigned long long)c2 * 0xCD9E8D57u;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c0 = n0; c1 = (uint32_t)p1; c2 = n2; c3 = (uint32_t)p0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return make_uint4(c0, c1, c2, c3);
}

// ---------------------------------------------------------------------------
// per-lane state
// ---------------------------------------------------------------------------
template <typename R> struct Lane {
  R l[3];         // position inside the current voxel, cm, in [0, d]
  R w[3];         // direction
  R E;            // kinetic energy, MeV
  R nd, nn;       // remaining delta / nuclear interaction lengths (mean free paths)
  R lacc;         // accumulated mass path for scattering, g/cm^2
  R lg;           // log2(lacc) (unused while lacc == 0)
  int32_t ix, iy, iz;
  int32_t v;      // linear voxel index
  int32_t hu;     // HU of the current voxel (clamped LUT index)
  int32_t vac;    // current voxel outside the external mask
  uint32_t b;     // next Philox block
  uint32_t h;     // history index within the spot
  int32_t spot;
  int32_t fate;   // kAlive while transported
  uint32_t nsteps;
  int32_t acc_v;  // merged tally: voxel and energy not yet added
  long long acc;
};

// per-lane totals reduced at kernel end
struct LaneCounters {
  unsigned long long esc, nuc, cut;
  unsigned long long out;  // deposits outside the spot's box (influence calculations)
  uint32_t hist, steps, delta, nuc_ev, escapes, misses, atomics;
};

// geometry of the phase a lane is in
template <typename R> struct Geo {
  const int16_t *hu;
  const uint8_t *mask;
  unsigned long long *tally;
  int32_t n[3];
  int32_t nxy;
  R d[3];
  int32_t lut;  // index of the phase's LUT in the launch's LUT array
};

// Where a lane's deposits go:
//   kTallyGrid  the phase tally (one global atomic per voxel visit)
//   kTallyBox   the spot's box tally (influence calculations); deposits
//               outside the box are only counted
//   kTallyCore  inside the spot's core: the block's LDS copy of the core
//               (flushed into the phase tally when the block is done with the
//               spot); outside it: the phase tally.  The core is a box of
//               the grid (a slice core of a beam along a grid axis)
//   kTallySlice kTallyCore with a slice core whose windows follow an
//               oblique beam (SliceCore)
//   kTallyBoxCore  kTallyBox whose core window (inside the box) adds into
//               the block's LDS copy (flushed into the box tally)
//   kTallyBoxSlice kTallyBoxCore with a slice core inside the box
//   kTallyCoreLog, kTallySliceLog  kTallyCore, kTallySlice that also write
//               the address of every global atomic into a per-lane log
//               (measurement of the deposit address pattern; the tallies are
//               the same)
constexpr int kTallyGrid = 0, kTallyBox = 1, kTallyCore = 2, kTallyBoxCore = 3, kTallyCoreLog = 4,
              kTallySlice = 5, kTallySliceLog = 6, kTallyBoxSlice = 7;

template <int TM>
constexpr bool kPhaseCore = TM == kTallyCore || TM == kTallyCoreLog || TM == kTallySlice || TM == kTallySliceLog;
template <int TM>
constexpr bool kLogged = TM == kTallyCoreLog || TM == kTallySliceLog;

// the box a lane's spot tallies into (kTallyBox: global, kTallyCore: LDS);
// kTallyBoxCore: the box (global) and its core window (LDS)
struct BoxLane {
  unsigned long long *base;  // entry 0 of the box
  int32_t lo[3], n[3];
  unsigned long long *core;  // kTallyBoxCore: entry 0 of the core window
  int32_t clo[3], cn[3];     // kTallyBoxCore: window corner (grid voxels) and size
  // kTallyCoreLog: entry n of this lane is log[n * log_stride + log_lane], n < log_cap
  unsigned long long *log;
  uint32_t log_cap, log_stride, log_lane;
  // kTallySlice, kTallySliceLog, kTallyBoxSlice: the spot's slice core
  // (SliceCore; sn = 0: none)
  int32_t sd, sa, se, sj0, sn, swa, swe, scells;
  int32_t sA[2], sB[2], smin[2], smax[2];
};

// corner of a slice-core window along one axis at slice j (SliceCore)
__device__ __forceinline__ int32_t slice_corner(int32_t A, int32_t Bs, int32_t j, int32_t mn, int32_t mx) {
  const int32_t c = (A + Bs * j) >> 16;
  return c < mn ? mn : (c > mx ? mx : c);
}

// physics tables per node i: (R, mu_delta, omega^2, dl2 / (R_{i+1} - R_i)),
// linear in log2 E between nodes; the last entry is the inverse slope of R
// against log2 E on the interval above the node (0 at the top node)
template <typename R> struct Tab {
  const typename M<R>::R4 *t;  // kNtab entries (LDS or global)
  R l2e0, inv_dl2, dl2;
};

// Axis selection on values, never through a pointer: a select of addresses
// into the lane state would keep that state out of registers.
template <typename T>
__device__ __forceinline__ T pick3(T x0, T x1, T x2, int k) {
  return k == 0 ? x0 : (k == 1 ? x1 : x2);
}
template <typename T>
__device__ __forceinline__ void set3(T &x0, T &x1, T &x2, int k, T v) {
  x0 = k == 0 ? v : x0;
  x1 = k == 1 ? v : x1;
  x2 = k == 2 ? v : x2;
}

// core entry of the lane's voxel in the slice core of B, or -1
template <typename R>
__device__ __forceinline__ int32_t slice_entry(const Lane<R> &L, const BoxLane &B) {
  const int32_t j = pick3(L.ix, L.iy, L.iz, B.sd) - B.sj0;
  if ((uint32_t)j < (uint32_t)B.sn) {
    const int32_t x = pick3(L.ix, L.iy, L.iz, B.sa) - slice_corner(B.sA[0], B.sB[0], j, B.smin[0], B.smax[0]);
    const int32_t y = pick3(L.ix, L.iy, L.iz, B.se) - slice_corner(B.sA[1], B.sB[1], j, B.smin[1], B.smax[1]);
    if ((uint32_t)x < (uint32_t)B.swa && (uint32_t)y < (uint32_t)B.swe) return j * B.scells + x + B.swa * y;
  }
  return -1;
}

// Pointers that reach a kernel through device memory (tables of targets,
// geometry in LDS) are generic to the compiler, which then emits flat
// instructions; on CDNA those also count against the LDS wait counter, so an
// LDS table read after a tally atomic would wait for the atomic to complete.
// Tallies, HU grids and masks live in device memory: address them as global.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T *as_global(T *p) {
  return (__attribute__((address_space(1))) T *)p;
}

__device__ __forceinline__ void atomic_add_u64(unsigned long long *p, unsigned long long v) {
  __hip_atomic_fetch_add(as_global(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// kTallyCoreLog: the address of the lane's n-th global atomic
__device__ __forceinline__ void log_atomic(const BoxLane &B, uint32_t n, const unsigned long long *p) {
  if (n < B.log_cap) as_global(B.log)[(size_t)n * B.log_stride + B.log_lane] = (unsigned long long)p;
}

// ---------------------------------------------------------------------------
// table lookups
// ---------------------------------------------------------------------------
template <typename R> struct Lookup { R R_, mud, om2, f, islope; int i; };

template <typename R>
__device__ __forceinline__ Lookup<R> lookup(const Tab<R> &T, R E) {
  const R x = (M<R>::log2(E) - T.l2e0) * T.inv_dl2;
  int i = (int)x;  // x >= 0 for E >= E_lo
  i = i < 0 ? 0 : (i > kNtab - 2 ? kNtab - 2 : i);
  const R f = x - (R)i;
  const auto a = T.t[i], b = T.t[i + 1];
  Lookup<R> o;
  o.R_ = a.x + f * (b.x - a.x);
  o.mud = a.y + f * (b.y - a.y);
  o.om2 = a.z + f * (b.z - a.z);
  o.f = f;
  o.islope = a.w;
  o.i = i;
  return o;
}

// exact inverse of the piecewise-linear range table; Rn < R(E) so the
// interval is at or below the current node i
template <typename R>
__device__ __forceinline__ R range_inverse(const Tab<R> &T, R Rn, int i) {
  if (!(Rn > (R)0)) return (R)kElo;
  int lo = i;
  R rlo = T.t[lo].x;
  while (lo > 0 && rlo > Rn) {
    --lo;
    rlo = T.t[lo].x;
  }
  const R rhi = T.t[lo + 1].x;
  const R f = M<R>::div(Rn - rlo, rhi - rlo);
  return M<R>::exp2(T.l2e0 + T.dl2 * ((R)lo + f));
}

template <typename R> struct Kin { R beta2, pbc, b2g2, g; };

template <typename R>
__device__ __forceinline__ Kin<R> kinematics(R E) {
  using MM = M<R>;
  const R tau = E * (R)(1.0 / kMp);
  Kin<R> k;
  k.g = (R)1 + tau;
  k.b2g2 = tau * (tau + (R)2);  // (beta gamma)^2
  const R ig = MM::rcp(k.g);
  k.beta2 = k.b2g2 * ig * ig;
  k.pbc = (R)kMp * k.b2g2 * ig;  // p beta c = (pc)^2 / E_total
  return k;
}

template <typename R>
__device__ __forceinline__ R tmax_of(const Kin<R> &k) {
  const R r = (R)(kMe / kMp);
  return M<R>::div((R)(2.0 * kMe) * k.b2g2, (R)1 + (R)2 * k.g * r + r * r);
}

// Highland projected-angle variance: theta^2(L) = A L c(L)^2 with
// A = (13.6 / p beta c)^2 / X0 and c(L) = 1 + 0.038 ln(L / (X0 beta^2)).
// ln L is carried from step to step (lg = log2 L of the accumulated path).
template <typename R> struct Highland { R A, lb; };

template <typename R>
__device__ __forceinline__ Highland<R> highland_at(const Kin<R> &k) {
  Highland<R> h;
  const R a = (R)13.6 * M<R>::rcp(k.pbc);
  h.A = a * a * (R)(1.0 / kX0);
  h.lb = M<R>::log2((R)kX0 * k.beta2);
  return h;
}

template <typename R>
__device__ __forceinline__ R highland2(const Highland<R> &h, R L, R lg) {
  if (!(L > (R)0)) return (R)0;
  const R c = (R)1 + (R)(0.038 * 0.69314718055994530942) * (lg - h.lb);
  return h.A * L * c * c;
}

// polar rotation of the unit direction w by (theta, phi = 2 pi u_phi)
template <typename R>
__device__ __forceinline__ void rotate(R w[3], R theta, R u_phi) {
  R ct, st;
  if constexpr (sizeof(R) == 4) {
    if (theta < 0.5f) {  // Taylor series: relative error below 1e-8 here
      const float t2 = theta * theta;
      st = theta * (1.0f - t2 * (1.0f / 6.0f) * (1.0f - t2 * (1.0f / 20.0f) * (1.0f - t2 * (1.0f / 42.0f))));
      ct = 1.0f - t2 * 0.5f * (1.0f - t2 * (1.0f / 12.0f) * (1.0f - t2 * (1.0f / 30.0f) * (1.0f - t2 * (1.0f / 56.0f))));
    } else {
      ct = __builtin_amdgcn_cosf(theta * 0.15915494309189533577f);
      st = __builtin_amdgcn_sinf(theta * 0.15915494309189533577f);
    }
  } else {
    ct = ::cos(theta);
    st = ::sin(theta);
  }
  const R cp = M<R>::cos_rev(u_phi), sp = M<R>::sin_rev(u_phi);
  const R a = w[0], b = w[1], c = w[2];
  const R den2 = a * a + b * b;
  R na, nb, nc;
  if (den2 < (R)1e-20) {
    na = st * cp;
    nb = st * sp;
    nc = (c >= (R)0 ? (R)1 : (R)-1) * ct;
  } else {
    const R den = M<R>::sqrt(den2);
    const R inv = M<R>::div((R)1, den);
    na = a * ct + st * (a * c * cp - b * sp) * inv;
    nb = b * ct + st * (b * c * cp + a * sp) * inv;
    nc = c * ct - st * cp * den;
  }
  R nn = na * na + nb * nb + nc * nc;
  R inv;
  if constexpr (sizeof(R) == 4) inv = __builtin_amdgcn_rsqf(nn);
  else inv = 1.0 / ::sqrt(nn);
  w[0] = na * inv;
  w[1] = nb * inv;
  w[2] = nc * inv;
}

template <typename R>
__device__ __forceinline__ int clamp_hu(int hu) {
  hu = hu < kHuMin ? kHuMin : (hu > kHuMax ? kHuMax : hu);
  return hu - kHuMin;
}

// ---------------------------------------------------------------------------
// source: sample the lateral offset and interaction lengths, enter the grid
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void start_history(Lane<R> &L, const SpotDev<R> &sp, int32_t spot,
                                              uint32_t h, const Geo<R> &G, uint32_t k0, uint32_t k1,
                                              LaneCounters &C) {
  const uint4 x = philox(0u, h, (uint32_t)spot, 0u, k0, k1);
  const R u0 = M<R>::uni(x.x), u1 = M<R>::uni(x.y), u2 = M<R>::uni(x.z), u3 = M<R>::uni(x.w);
  const R rad = M<R>::sqrt((R)-2 * ((R)0.69314718055994530942 * M<R>::log2(u0)));
  const R gx = rad * M<R>::cos_rev(u1), gy = rad * M<R>::sin_rev(u1);
  L.nn = (R)-0.69314718055994530942 * M<R>::log2(u2);
  L.nd = (R)-0.69314718055994530942 * M<R>::log2(u3);
  L.E = sp.E;
  L.h = h;
  L.spot = spot;
  L.b = 1u;
  L.lacc = (R)0;
  L.lg = (R)0;
  L.nsteps = 0;
  L.acc_v = -1;
  L.acc = 0;
  C.hist += 1;
  const R a = sp.sigma * gx, bb = sp.sigma * gy;
  R p[3], r[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    L.w[k] = sp.w[k];
    p[k] = sp.c[k] + a * sp.u[k] + bb * sp.v[k];
  }
  // slab method on [0, n d)
  R tn = -M<R>::inf(), tf = M<R>::inf();
  int an = -1;
  bool missed = false;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const R ext = (R)G.n[k] * G.d[k];
    if (L.w[k] != (R)0) {
      const R iw = M<R>::div((R)1, L.w[k]);
      const R t1 = ((R)0 - p[k]) * iw, t2 = (ext - p[k]) * iw;
      const R lo = t1 < t2 ? t1 : t2, hi = t1 < t2 ? t2 : t1;
      if (lo > tn) { tn = lo; an = k; }
      if (hi < tf) tf = hi;
    } else if (p[k] < (R)0 || p[k] >= ext) {
      missed = true;
    }
  }
  if (an < 0 || !(tn < tf)) missed = true;
  // one exit path: every field is written exactly once below
  int idx[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    r[k] = p[k] + tn * L.w[k];
    int i;
    R l;
    if (k == an) {
      i = L.w[k] > (R)0 ? 0 : G.n[k] - 1;
      l = L.w[k] > (R)0 ? (R)0 : G.d[k];
    } else {
      i = (int)floor(M<R>::div(r[k], G.d[k]));
      i = i < 0 ? 0 : (i > G.n[k] - 1 ? G.n[k] - 1 : i);
      l = r[k] - (R)i * G.d[k];
    }
    idx[k] = missed ? 0 : i;
    L.l[k] = missed ? p[k] : l;
  }
  L.ix = idx[0];
  L.iy = idx[1];
  L.iz = idx[2];
  const int v = idx[0] + G.n[0] * (idx[1] + G.n[1] * idx[2]);
  L.v = missed ? -1 : v;
  const int hu = as_global(G.hu)[v];  // v is in range in both cases (0 when missed)
  L.hu = clamp_hu<R>(hu);
  L.vac = (G.mask && !missed) ? (as_global(G.mask)[v] == 0) : 0;
  L.fate = missed ? kMissed : kAlive;
  if (missed) {
    C.esc += (unsigned long long)M<R>::q(L.E);
    C.misses += 1;
  }
}

// Tally key of a deposit.  kTallyGrid: the voxel index; kTallyBox: the
// box-local entry, -2 outside the box; kTallyCore, kTallySlice: -3 - (core
// entry) inside the core, else the voxel index; kTallyBoxCore: -2 outside the box,
// -3 - (window-local entry) inside the window, else the box-local entry.  The
// lane is still in the voxel of the step.
template <typename R, int TM>
__device__ __forceinline__ int32_t tally_key(const Lane<R> &L, const BoxLane &B, int32_t v) {
  if constexpr (TM == kTallyGrid) {
    return v;
  } else if constexpr (TM == kTallyCore || TM == kTallyCoreLog) {
    const int32_t x = L.ix - B.lo[0], y = L.iy - B.lo[1], z = L.iz - B.lo[2];
    const bool in = (uint32_t)x < (uint32_t)B.n[0] && (uint32_t)y < (uint32_t)B.n[1] &&
                    (uint32_t)z < (uint32_t)B.n[2];
    return in ? -3 - (x + B.n[0] * (y + B.n[1] * z)) : v;
  } else if constexpr (TM == kTallySlice || TM == kTallySliceLog) {
    const int32_t c = slice_entry(L, B);
    return c >= 0 ? -3 - c : v;
  } else if constexpr (TM == kTallyBoxSlice) {
    const int32_t x = L.ix - B.lo[0], y = L.iy - B.lo[1], z = L.iz - B.lo[2];
    if (!((uint32_t)x < (uint32_t)B.n[0] && (uint32_t)y < (uint32_t)B.n[1] &&
          (uint32_t)z < (uint32_t)B.n[2]))
      return -2;
    const int32_t c = slice_entry(L, B);
    return c >= 0 ? -3 - c : x + B.n[0] * (y + B.n[1] * z);
  } else if constexpr (TM == kTallyBoxCore) {
    const int32_t x = L.ix - B.lo[0], y = L.iy - B.lo[1], z = L.iz - B.lo[2];
    if (!((uint32_t)x < (uint32_t)B.n[0] && (uint32_t)y < (uint32_t)B.n[1] &&
          (uint32_t)z < (uint32_t)B.n[2]))
      return -2;
    const int32_t cx = L.ix - B.clo[0], cy = L.iy - B.clo[1], cz = L.iz - B.clo[2];
    const bool in_core = (uint32_t)cx < (uint32_t)B.cn[0] && (uint32_t)cy < (uint32_t)B.cn[1] &&
                         (uint32_t)cz < (uint32_t)B.cn[2];
    return in_core ? -3 - (cx + B.cn[0] * (cy + B.cn[1] * cz)) : x + B.n[0] * (y + B.n[1] * z);
  } else {
    static_assert(TM == kTallyBox, "tally mode");
    const int32_t x = L.ix - B.lo[0], y = L.iy - B.lo[1], z = L.iz - B.lo[2];
    const bool in = (uint32_t)x < (uint32_t)B.n[0] && (uint32_t)y < (uint32_t)B.n[1] &&
                    (uint32_t)z < (uint32_t)B.n[2];
    return in ? x + B.n[0] * (y + B.n[1] * z) : -2;
  }
}

template <typename R, int TM>
__device__ __forceinline__ void commit_acc(const Lane<R> &L, const Geo<R> &G, const BoxLane &B,
                                           LaneCounters &C) {
  if (L.acc == 0) return;
  if constexpr (TM == kTallyBox) {
    if (L.acc_v < 0) {
      C.out += (unsigned long long)L.acc;
      return;
    }
    atomic_add_u64(&B.base[L.acc_v], (unsigned long long)L.acc);
  } else if constexpr (kPhaseCore<TM>) {
    if (L.acc_v <= -3) {  // LDS: the block's copy of the core
      __hip_atomic_fetch_add(&B.base[-3 - L.acc_v], (unsigned long long)L.acc, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
      return;
    }
    atomic_add_u64(&G.tally[L.acc_v], (unsigned long long)L.acc);
    if constexpr (kLogged<TM>) log_atomic(B, C.atomics, &G.tally[L.acc_v]);
  } else if constexpr (TM == kTallyBoxCore || TM == kTallyBoxSlice) {
    if (L.acc_v <= -3) {  // LDS: the block's copy of the core window
      __hip_atomic_fetch_add(&B.core[-3 - L.acc_v], (unsigned long long)L.acc, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
      return;
    }
    if (L.acc_v == -2) {
      C.out += (unsigned long long)L.acc;
      return;
    }
    atomic_add_u64(&B.base[L.acc_v], (unsigned long long)L.acc);
  } else {
    atomic_add_u64(&G.tally[L.acc_v], (unsigned long long)L.acc);
  }
  C.atomics += 1;
}

template <typename R, int TM = kTallyGrid>
__device__ __forceinline__ void flush_tally(Lane<R> &L, const Geo<R> &G, LaneCounters &C,
                                            const BoxLane &B = BoxLane{}) {
  commit_acc<R, TM>(L, G, B, C);
  L.acc = 0;
  L.acc_v = -1;
}

// consecutive deposits into the same voxel are merged in registers: at most
// one atomic per voxel visit
template <typename R, int TM>
__device__ __forceinline__ void add_tally(Lane<R> &L, const Geo<R> &G, const BoxLane &B, int32_t v,
                                          long long dep, LaneCounters &C) {
  if (dep == 0) return;
  const int32_t key = tally_key<R, TM>(L, B, v);
  if (key != L.acc_v) {
    commit_acc<R, TM>(L, G, B, C);
    L.acc_v = key;
    L.acc = dep;
  } else {
    L.acc += dep;
  }
}

template <typename R>
__device__ __forceinline__ void trace_out(TraceRec *rec, int n, int max_rec, int cause, int voxel,
                                          const Lane<R> &L, const Geo<R> &G, R s, long long dep,
                                          R t_delta) {
  if (n >= max_rec) return;
  TraceRec &o = rec[n];
  o.cause = cause;
  o.voxel = voxel;
  o.fate = L.fate;
  o.block = L.b;
  o.s = (double)s;
  o.E = L.fate == kStopped ? 0.0 : (double)L.E;
  const int idx[3] = {L.ix, L.iy, L.iz};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    o.r[k] = (double)idx[k] * (double)G.d[k] + (double)L.l[k];
    o.w[k] = (double)L.w[k];
  }
  o.n_delta = (double)L.nd;
  o.n_nuc = (double)L.nn;
  o.l_acc = (double)L.lacc;
  o.dep = dep;
  o.t_delta = (double)t_delta;
}

// ---------------------------------------------------------------------------
// one condensed-history step
// ---------------------------------------------------------------------------
template <typename R, bool TRACE, int TM = kTallyGrid>
__device__ __forceinline__ void step(Lane<R> &L, const Geo<R> &G, const Tab<R> &T,
                                     const typename M<R>::R2 *lut, uint32_t k0, uint32_t k1,
                                     uint32_t flags, LaneCounters &C, TraceRec *rec, int max_rec,
                                     const BoxLane &B = BoxLane{}) {
  using MM = M<R>;
  const R LN2 = (R)0.69314718055994530942;
  // 1. material
  const auto m = lut[L.hu];
  const R rho = m.x, rsp = m.y;
  const bool vac = L.vac != 0;

  // 2. boundary distance (lowest axis wins ties) and prefetch of the neighbour
  R dg = MM::inf();
  int ax = -1;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const R wk = L.w[k];
    if (wk != (R)0) {
      R t = MM::div(wk > (R)0 ? (G.d[k] - L.l[k]) : -L.l[k], wk);
      t = t < (R)0 ? (R)0 : t;
      if (t < dg) { dg = t; ax = k; }
    }
  }
  const bool ax_pos = pick3(L.w[0], L.w[1], L.w[2], ax) > (R)0;
  const int idx_ax = pick3(L.ix, L.iy, L.iz, ax);
  const int n_ax = pick3(G.n[0], G.n[1], G.n[2], ax);
  const int nb_idx = idx_ax + (ax_pos ? 1 : -1);
  const bool nb_in = nb_idx >= 0 && nb_idx < n_ax;
  const int stride = pick3(1, G.n[0], G.nxy, ax);
  const int v_nb = L.v + (ax_pos ? stride : -stride);
  int hu_nb = 0, mask_nb = 1;
  if (nb_in) {
    hu_nb = as_global(G.hu)[v_nb];
    if (G.mask) mask_nb = as_global(G.mask)[v_nb];
  }

  // 3-4. physics limits; priority on ties stop > geo > delta > nuclear > phys
  R s = dg, Rr = 0, mud = 0, om2 = 0, mun = 0, tf = 0, tis = 0;
  int ti = 0;
  int cause = kGeo;
  if (!vac) {
    const Lookup<R> lk = lookup(T, L.E);
    Rr = lk.R_;
    mud = (flags & kNoDelta) ? (R)0 : lk.mud;
    om2 = lk.om2;
    ti = lk.i;
    tf = lk.f;
    tis = lk.islope;
    mun = (!(flags & kNoNuclear) && L.E >= (R)kEn) ? (R)kMuN : (R)0;
    const R inv_rsp = MM::rcp(rsp);
    const R s_stop = (flags & kFrozen) ? MM::inf() : (rsp > (R)0 ? Rr * inv_rsp : MM::inf());
    const R s_phys = rsp > (R)0 ? MM::fmax((R)kEpsR * Rr, (R)kSfloor) * inv_rsp : MM::inf();
    const R cd = mud * rsp, cn = mun * rho;
    R d_d = cd > (R)0 ? MM::div(L.nd, cd) : MM::inf();
    R d_n = cn > (R)0 ? MM::div(L.nn, cn) : MM::inf();
    d_d = d_d < (R)0 ? (R)0 : d_d;
    d_n = d_n < (R)0 ? (R)0 : d_n;
    s = s_stop;
    cause = kStop;
    if (dg < s) { s = dg; cause = kGeo; }
    if (d_d < s) { s = d_d; cause = kDelta; }
    if (d_n < s) { s = d_n; cause = kNuc; }
    if (s_phys < s) { s = s_phys; cause = kPhys; }
  }
  // one fresh block per step
  const uint4 x = philox(L.b, L.h, (uint32_t)L.spot, 0u, k0, k1);
  L.b += 1u;

  // 5. move; a boundary step lands exactly on the face
#pragma unroll
  for (int k = 0; k < 3; ++k) L.l[k] += s * L.w[k];
  const R d_ax = pick3(G.d[0], G.d[1], G.d[2], ax);
  if (cause == kGeo) set3(L.l[0], L.l[1], L.l[2], ax, ax_pos ? d_ax : (R)0);

  const R E_pre = L.E;
  long long dep = 0;
  R t_delta = 0;
  const int v_step = L.v;
  if (!vac) {
    // 6. continuous loss with Gaussian soft straggling
    if (!(flags & kFrozen)) {
      if (cause == kStop) {
        L.fate = kStopped;
      } else {
        const R sw = rsp * s;
        const R g = (flags & kNoStraggling)
                        ? (R)0
                        : MM::sqrt((R)-2 * (LN2 * MM::log2(MM::uni(x.x)))) * MM::cos_rev(MM::uni(x.y));
        // mean loss: the exact inverse of the piecewise-linear range table.
        // A step that ends in the log E interval it starts in moves log2 E
        // down by y = sw dl2 / (R_{i+1} - R_i) exactly, so E' = E 2^-y; the
        // loss is formed from y directly rather than as E - R^-1(R(E) - sw),
        // whose working-precision rounding of the table coordinate is large
        // against the loss of a step through air.
        const R y = sw * tis;
        const R d_mean = y <= T.dl2 * tf ? L.E * MM::one_minus_exp2_neg(y)
                                         : L.E - range_inverse(T, Rr - sw, ti);
        R dE = d_mean + MM::sqrt(om2 * sw) * g;
        dE = dE < (R)0 ? (R)0 : (dE > L.E ? L.E : dE);
        const R En = L.E - dE;
        if (En <= (R)kElo) L.fate = kStopped;
        else L.E = En;
      }
    }
    // 7. interaction lengths with pre-step coefficients
    L.nd -= mud * rsp * s;
    L.nn -= mun * rho * s;
    if (cause == kDelta) L.nd = (R)0;
    if (cause == kNuc) L.nn = (R)0;
    // 8. telescoping Highland at the pre-step energy
    const Highland<R> hp = highland_at(kinematics(E_pre));
    const R l_new = L.lacc + rho * s;
    const R lg_new = l_new > (R)0 ? MM::log2(l_new) : (R)0;
    R th2 = highland2(hp, l_new, lg_new) - highland2(hp, L.lacc, L.lg);
    th2 = th2 < (R)0 ? (R)0 : th2;
    L.lacc = l_new;
    L.lg = lg_new;
    if (L.fate == kAlive && !(flags & kNoMcs) && th2 > (R)0) {
      const R theta = MM::sqrt(th2) * MM::sqrt((R)-2 * (LN2 * MM::log2(MM::uni(x.z))));
      rotate(L.w, theta, MM::uni(x.w));
    }
    // 9. tally by telescoping fixed-point energy
    if (L.fate == kStopped) {
      dep = MM::q(E_pre);
      C.cut += (unsigned long long)MM::q(E_pre);
    } else {
      dep = MM::q(E_pre) - MM::q(L.E);
    }
    // 10. events at the step end
    if (L.fate == kAlive && cause == kDelta) {
      const Kin<R> k = kinematics(L.E);
      const R tmax = tmax_of(k);
      if (tmax > (R)kTcut) {
        const R a = (R)(1.0 / kTcut), bt = (R)(1.0 / kTcut) - MM::div((R)1, tmax);
        const R cb = MM::div(k.beta2, tmax);
        R T_d = (R)kTcut;
        // acceptance is >= 1/2 per trial; the bound only guarantees termination
        for (int trial = 0; trial < 4096; ++trial) {
          const uint4 y = philox(L.b, L.h, (uint32_t)L.spot, 0u, k0, k1);
          L.b += 1u;
          const R t1 = MM::div((R)1, a - MM::uni(y.x) * bt);
          if (MM::uni(y.y) < (R)1 - cb * t1) { T_d = t1; break; }
          const R t2 = MM::div((R)1, a - MM::uni(y.z) * bt);
          if (MM::uni(y.w) < (R)1 - cb * t2) { T_d = t2; break; }
        }
        const R cap = L.E - (R)kElo;
        T_d = T_d > cap ? cap : T_d;
        t_delta = T_d;
        C.delta += 1;
        if (!(flags & kFrozen)) {
          const R En = L.E - T_d;
          dep += MM::q(L.E) - MM::q(En);
          L.E = En;
          if (L.E <= (R)kElo) {
            dep += MM::q(L.E);
            C.cut += (unsigned long long)MM::q(L.E);
            L.fate = kStopped;
          }
        }
      }
      const uint4 y = philox(L.b, L.h, (uint32_t)L.spot, 0u, k0, k1);
      L.b += 1u;
      L.nd = -LN2 * MM::log2(MM::uni(y.x));
    } else if (L.fate == kAlive && cause == kNuc) {
      C.nuc += (unsigned long long)MM::q(L.E);
      C.nuc_ev += 1;
      L.fate = kNuclear;
    }
  }
  // Take the prefetched neighbour (HU, mask) here, on every path and before
  // this step's tally atomic.  Vector memory operations complete in order, so
  // a wait for the prefetch placed after the atomic (the compiler puts it
  // before the first use, in the crossing below) also waited for the atomic's
  // round trip to the memory side; here it covers only the previous step's
  // atomic, issued a whole step earlier.  The empty asm emits nothing; its
  // register operands make the value needed at this point.  (dep is 0 in
  // vacuum, where add_tally does nothing.)
  asm volatile("" ::"v"(hu_nb), "v"(mask_nb));
  add_tally<R, TM>(L, G, B, v_step, dep, C);
  C.steps += 1;
  L.nsteps += 1;
  // 11. boundary crossing
  if (L.fate == kAlive && cause == kGeo) {
    if (!nb_in) {
      C.esc += (unsigned long long)MM::q(L.E);
      C.escapes += 1;
      L.fate = kEscaped;
    } else {
      set3(L.ix, L.iy, L.iz, ax, nb_idx);
      set3(L.l[0], L.l[1], L.l[2], ax, ax_pos ? (R)0 : d_ax);
      L.v = v_nb;
      L.hu = clamp_hu<R>(hu_nb);
      L.vac = mask_nb == 0;
    }
  }
  if (L.fate == kAlive && L.nsteps >= kMaxSteps) {  // safety valve, never reached by valid input
    C.esc += (unsigned long long)MM::q(L.E);
    C.escapes += 1;
    L.fate = kEscaped;
  }
  if constexpr (TRACE) trace_out(rec, (int)L.nsteps, max_rec, cause, v_step, L, G, s, dep, t_delta);
}

}  // namespace pmc
