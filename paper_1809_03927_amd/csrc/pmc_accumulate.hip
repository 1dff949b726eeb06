// Deformable dose accumulation by energy/mass transfer (Sec. 2.D.2, Eqs. (2),
// (4)-(6)) with DVFs stored as in App. B (Eqs. (7)-(8)).
//
//  emtm_push    one thread per source voxel: its n^3 subvoxel centres are
//               mapped to the reference grid (trilinear interpolation of the
//               DVF translations, FP64); the voxel's energy (tally, as two
//               32-bit halves) and mass units (round(rho 2^32)) are added,
//               once per subvoxel, to the reference voxel each centre lands
//               in.  The thread counts its subvoxels per reference voxel in a
//               private LDS window of 4x4x4 voxels (16-bit counts) around the
//               first one, and adds count x energy and count x mass with one
//               set of device atomics per voxel it reached.
//  emtm_ratio   dose_i += sum E / sum M (Eq. (5)) per reference voxel, in
//               Gy per history, added in source order (Eq. (2)).
//  emtm_mask    keeps the dose where the reference voxel centre lies in the
//               grid box of every DVF.
//  dim_pull     dose interpolation (Eq. (3)): one thread per reference voxel
//               maps its n^3 subvoxel centres to the source phase and adds
//               the average of the source dose sampled there.
//  dvf_points   the full field of App. B (Eqs. (8), (7)), one thread per grid
//               point.
//
// Every floating-point decision (which reference voxel a centre lands in)
// equals that of a plain FP64 evaluation of the formulas in their written
// order (no contraction), and every sum is an integer sum, so the result does
// not depend on the schedule.
//
// Axis-aligned DVF grids (row (1,0,0), column (0,1,0), so depth (0,0,1)):
// the grid coordinate along an axis is then the point's own coordinate minus
// the start over the spacing, exactly (x*1 = x, the other terms are signed
// zeros, which change no decision below), so each axis is evaluated once per
// subvoxel row (z: once per voxel, kept in LDS).  With z innermost, the
// x- and y-interpolated translations of a DVF cell are reused while the
// subvoxels stay in that cell; a wave's lanes share z, so the reload is
// wave-uniform.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "pmc_internal.hpp"

namespace pmc {

namespace {

constexpr int kMaxSub = 16;
constexpr int kWin = 4;                              // window offsets -1..+2 per axis
constexpr int kWinCells = kWin * kWin * kWin;

// log2 of the counts per 32-bit window word: four 8-bit counts while a voxel
// has at most 255 subvoxels (n <= 6), else two 16-bit counts (n^3 <= 4096).
__host__ __device__ __forceinline__ int win_lg(int n) { return n * n * n <= 255 ? 2 : 1; }

template <class G>
__device__ __forceinline__ bool dvf_coords(const G &d, double px, double py, double pz, double g[3]) {
  const double rx = px - d.start[0], ry = py - d.start[1], rz = pz - d.start[2];
  const double ax[3][3] = {{d.u[0], d.u[1], d.u[2]}, {d.v[0], d.v[1], d.v[2]}, {d.w[0], d.w[1], d.w[2]}};
  bool inside = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    g[a] = (rx * ax[a][0] + ry * ax[a][1] + rz * ax[a][2]) / d.sp[a];
    inside = inside && g[a] >= 0.0 && g[a] <= (double)(d.n[a] - 1);
  }
  return inside;
}

// A rigid 4x4 matrix (rows 0..2) applied to a point: m[a][0] x + m[a][1] y +
// m[a][2] z + m[a][3], summed in that order.
__device__ __forceinline__ void rigid(const double m[12], const double p[3], double out[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) out[a] = m[4 * a] * p[0] + m[4 * a + 1] * p[1] + m[4 * a + 2] * p[2] + m[4 * a + 3];
}

// T(r) of Eq. (1): M_post (M_pre r + the trilinear interpolation (x, then y,
// then z) of the translations of the 8 grid points around r); without the
// rigid matrices r plus that interpolation.  False outside the grid.
__device__ __forceinline__ bool dvf_map(const DvfDev &d, double px, double py, double pz, double q[3]) {
  double g[3];
  if (!dvf_coords(d, px, py, pz, g)) return false;
  int b[3];
  double f[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    int i = (int)floor(g[a]);
    if (i > d.n[a] - 2) i = d.n[a] - 2;
    b[a] = i;
    f[a] = g[a] - (double)i;
  }
  const long long sx = 3, sy = 3LL * d.n[0], sz = 3LL * d.n[0] * d.n[1];
  const double *c = d.delta + b[0] * sx + b[1] * sy + b[2] * sz;
  const double p[3] = {px, py, pz};
  double base[3] = {px, py, pz};
  if (d.has_pre) rigid(d.pre, p, base);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double d000 = c[k], d100 = c[sx + k], d010 = c[sy + k], d110 = c[sx + sy + k];
    const double d001 = c[sz + k], d101 = c[sx + sz + k], d011 = c[sy + sz + k], d111 = c[sx + sy + sz + k];
    const double c00 = d000 + f[0] * (d100 - d000);
    const double c10 = d010 + f[0] * (d110 - d010);
    const double c01 = d001 + f[0] * (d101 - d001);
    const double c11 = d011 + f[0] * (d111 - d011);
    const double c0 = c00 + f[1] * (c10 - c00);
    const double c1 = c01 + f[1] * (c11 - c01);
    q[k] = base[k] + (c0 + f[2] * (c1 - c0));
  }
  if (d.has_post) {
    const double r[3] = {q[0], q[1], q[2]};
    rigid(d.post, r, q);
  }
  return true;
}

__device__ __forceinline__ void add_u64(unsigned long long *p, unsigned long long v) {
  __hip_atomic_fetch_add((__attribute__((address_space(1))) unsigned long long *)p, v, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
}

struct Deposit {
  unsigned long long t_hi, t_lo, mq;
};

__device__ __forceinline__ void deposit(const EmtmPush &a, const Deposit &d, int i, unsigned long long c) {
  if (d.t_hi) add_u64(a.e_hi + i, c * d.t_hi);
  if (d.t_lo) add_u64(a.e_lo + i, c * d.t_lo);
  add_u64(a.mass + i, c * d.mq);
}

// This thread's subvoxel counts per reference voxel: word k of the window at
// w[k * stride] holds the counts of window cells k 2^lg .. (k + 1) 2^lg - 1.
struct Window {
  uint32_t *w;
  int stride;  // threads of the block: word k of this thread's window at w[k * stride]
  int lg;
  int b[3];
  uint32_t touched;  // words holding counts
  bool set;
};

// Reference voxel of a mapped point q (Eq. (6): the voxel containing it);
// false outside the reference grid.  Along each axis the index is
// floor(RN(t / r)), t = q - origin, as a plain division gives it.  With
// a = t * rinv (rinv = RN(1/r)): |a - t/r| <= |t/r| (2^-52 + 2^-106) and
// |RN(t/r) - t/r| <= |t/r| 2^-53, so |a - RN(t/r)| < |a| 2^-50, below 2^-30
// while |a| < 2^20.  Then if a - floor(a) lies in [2^-30, 1 - 2^-30],
// RN(t/r) has the floor of a.  (That difference is exact except for
// -1/2 < a < 0, where floor(RN(t/r)) = -1 = floor(a) anyway.)  For
// |a| >= 2^20 both floors lie outside a grid of fewer than 2^20 voxels per
// axis.  Otherwise, a within 2^-30 of an integer (rare), the divisions
// decide.  Coordinates in mm give no subnormal quotients.
__device__ __forceinline__ bool ref_voxel(const EmtmPush &a, double qx, double qy, double qz, int t[3]) {
  const double tx = qx - a.rorg[0], ty = qy - a.rorg[1], tz = qz - a.rorg[2];
  const double ax = tx * a.rinv[0], ay = ty * a.rinv[1], az = tz * a.rinv[2];
  double kx = floor(ax), ky = floor(ay), kz = floor(az);
  const double ex = ax - kx, ey = ay - ky, ez = az - kz;
  constexpr double lo = 0x1p-30, hi = 1.0 - 0x1p-30;
  const bool sure = (ex >= lo) & (ex <= hi) & (ey >= lo) & (ey <= hi) & (ez >= lo) & (ez <= hi);
  if (!sure) {
    kx = floor(tx / a.rsp[0]);
    ky = floor(ty / a.rsp[1]);
    kz = floor(tz / a.rsp[2]);
  }
  if (!((kx >= 0.0) & (kx < (double)a.rnx) & (ky >= 0.0) & (ky < (double)a.rny) & (kz >= 0.0) &
        (kz < (double)a.rnz)))
    return false;
  t[0] = (int)kx;
  t[1] = (int)ky;
  t[2] = (int)kz;
  return true;
}

__device__ __forceinline__ void count(const EmtmPush &a, Window &win, const Deposit &d, const int t[3]) {
  if (a.n_sub == 1) {
    deposit(a, d, t[0] + a.rnx * (t[1] + a.rny * t[2]), 1);
    return;
  }
  const bool first = !win.set;
  win.b[0] = first ? t[0] - 1 : win.b[0];
  win.b[1] = first ? t[1] - 1 : win.b[1];
  win.b[2] = first ? t[2] - 1 : win.b[2];
  win.set = true;
  const unsigned dx = (unsigned)(t[0] - win.b[0]), dy = (unsigned)(t[1] - win.b[1]),
                 dz = (unsigned)(t[2] - win.b[2]);
  if (dx < kWin && dy < kWin && dz < kWin) {
    const unsigned c = dx + kWin * (dy + kWin * dz);
    const unsigned lg = (unsigned)win.lg;
    win.touched |= 1u << (c >> lg);
    __hip_atomic_fetch_add(win.w + (c >> lg) * win.stride, 1u << ((c & ((1u << lg) - 1u)) << (5u - lg)),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  } else {
    deposit(a, d, t[0] + a.rnx * (t[1] + a.rny * t[2]), 1);
  }
}

__device__ __forceinline__ void flush(const EmtmPush &a, Window &win, const Deposit &d) {
  const int per = 1 << win.lg, bits = 32 >> win.lg;
  const uint32_t field = (1u << bits) - 1u;
  while (win.touched) {
    const int k = __builtin_ctz(win.touched);
    win.touched &= win.touched - 1u;
    const uint32_t v = win.w[k * win.stride];
    win.w[k * win.stride] = 0;
    for (int h = 0; h < per; ++h) {
      const uint32_t c = (v >> (bits * h)) & field;
      if (!c) continue;
      const int e = per * k + h;
      const int x = win.b[0] + (e & 3), y = win.b[1] + ((e >> 2) & 3), z = win.b[2] + (e >> 4);
      deposit(a, d, x + a.rnx * (y + a.rny * z), c);
    }
  }
  win.set = false;
}

// Grid cell and fraction along one axis of the DVF grid (inside already checked).
__device__ __forceinline__ int cell(double g, int n, double &f) {
  int i = (int)floor(g);
  if (i > n - 2) i = n - 2;
  f = g - (double)i;
  return i;
}

// The n^3 subvoxel centres of voxel (ix, iy, iz) of a grid (origin org,
// spacing sp, mm) mapped by the DVF g: visit(qx, qy, qz) for every centre
// inside the DVF grid, x outermost, then y, then z.  ALIGNED (identity
// directions, no rigid matrices): the grid coordinate along an axis is exactly
// (coordinate - start) / spacing, so z is tabulated per voxel in this thread's
// LDS table (zf: fraction, zp: coordinate, zb: cell or -1 outside; n entries,
// stride B, the block size) and the x- then y-interpolated translations of a DVF cell are
// kept while the centres stay in it.
template <bool ALIGNED, int B, class Visit>
__device__ __forceinline__ void map_subvoxels(const DvfDev &g, const double *org, const double *sp, int n, int ix,
                                              int iy, int iz, const double *off, double *zf, double *zp, int *zb,
                                              int tid, Visit &&visit) {
  if (ALIGNED) {
    // z: coordinate, DVF cell and fraction of every subvoxel plane (cell -1
    // outside the grid)
    for (int sc = 0; sc < n; ++sc) {
      const double pz = org[2] + ((double)iz + off[sc]) * sp[2];
      const double gz = (pz - g.start[2]) / g.sp[2];
      double f = 0.0;
      int b = -1;
      if (gz >= 0.0 && gz <= (double)(g.n[2] - 1)) b = cell(gz, g.n[2], f);
      zf[sc * B + tid] = f;
      zp[sc * B + tid] = pz;
      zb[sc * B + tid] = b;
    }
    const long long sy = 3LL * g.n[0], sz = 3LL * g.n[0] * g.n[1];
    for (int sa = 0; sa < n; ++sa) {
      const double px = org[0] + ((double)ix + off[sa]) * sp[0];
      const double gx = (px - g.start[0]) / g.sp[0];
      if (!(gx >= 0.0 && gx <= (double)(g.n[0] - 1))) continue;
      double f0;
      const int b0 = cell(gx, g.n[0], f0);
      for (int sb = 0; sb < n; ++sb) {
        const double py = org[1] + ((double)iy + off[sb]) * sp[1];
        const double gy = (py - g.start[1]) / g.sp[1];
        if (!(gy >= 0.0 && gy <= (double)(g.n[1] - 1))) continue;
        double f1;
        const int b1 = cell(gy, g.n[1], f1);
        const double *col = g.delta + 3LL * b0 + sy * b1;
        // c0, c1: translations interpolated in x then y on the lower and
        // upper z plane of DVF cell layer cb; dc = c1 - c0
        int cb = -1;
        double c0[3], c1[3], dc[3];
        for (int sc = 0; sc < n; ++sc) {
          const int b2 = zb[sc * B + tid];
          if (b2 < 0) continue;
          const double f2 = zf[sc * B + tid];
          if (b2 != cb) {
            // z grows with sc, so the next layer is usually cb + 1, whose
            // lower plane is cb's upper plane: the same corners and
            // operations give the same c0
            const double *c = col + sz * b2;
            if (cb >= 0 && b2 == cb + 1) {
#pragma unroll
              for (int k = 0; k < 3; ++k) c0[k] = c1[k];
            } else {
#pragma unroll
              for (int k = 0; k < 3; ++k) {
                const double d000 = c[k], d100 = c[3 + k], d010 = c[sy + k], d110 = c[sy + 3 + k];
                const double c00 = d000 + f0 * (d100 - d000);
                const double c10 = d010 + f0 * (d110 - d010);
                c0[k] = c00 + f1 * (c10 - c00);
              }
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
              const double d001 = c[sz + k], d101 = c[sz + 3 + k], d011 = c[sz + sy + k],
                           d111 = c[sz + sy + 3 + k];
              const double c01 = d001 + f0 * (d101 - d001);
              const double c11 = d011 + f0 * (d111 - d011);
              c1[k] = c01 + f1 * (c11 - c01);
              dc[k] = c1[k] - c0[k];
            }
            cb = b2;
          }
          const double pz = zp[sc * B + tid];
          const double qx = px + (c0[0] + f2 * dc[0]);
          const double qy = py + (c0[1] + f2 * dc[1]);
          const double qz = pz + (c0[2] + f2 * dc[2]);
          visit(qx, qy, qz);
        }
      }
    }
  } else {
    for (int sa = 0; sa < n; ++sa) {
      const double px = org[0] + ((double)ix + off[sa]) * sp[0];
      for (int sb = 0; sb < n; ++sb) {
        const double py = org[1] + ((double)iy + off[sb]) * sp[1];
        for (int sc = 0; sc < n; ++sc) {
          const double pz = org[2] + ((double)iz + off[sc]) * sp[2];
          double q[3];
          if (!dvf_map(g, px, py, pz, q)) continue;
          visit(q[0], q[1], q[2]);
        }
      }
    }
  }
}

template <bool ALIGNED, int B>
__global__ void __launch_bounds__(B) emtm_push(EmtmPush a) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double off[kMaxSub];
  const int n = a.n_sub;
  const int tid = threadIdx.x;
  const int lg = win_lg(n);
  const int words = kWinCells >> lg;
  uint32_t *win_words = reinterpret_cast<uint32_t *>(smem);
  double *zf = reinterpret_cast<double *>(smem + sizeof(uint32_t) * words * B);
  double *zp = zf + (size_t)n * B;
  int *zb = reinterpret_cast<int *>(zp + (size_t)n * B);
  // subvoxel centre offsets (s + 1/2) / n, in voxels
  if (tid < n) off[tid] = ((double)tid + 0.5) / (double)n;
  for (int k = 0; k < words; ++k) win_words[k * B + tid] = 0;
  __syncthreads();
  Window win;
  win.w = win_words + tid;
  win.stride = B;
  win.lg = lg;
  win.touched = 0;
  win.set = false;
  const DvfDev &g = a.dvf;
  // grids hold at most 2^31 - 1 voxels
  const unsigned nvox = (unsigned)a.nx * (unsigned)a.ny * (unsigned)a.nz;
  const unsigned stride = gridDim.x * B;
  for (unsigned j = blockIdx.x * B + tid; j < nvox; j += stride) {
    double rho = 0.0;
    if (!a.mask || a.mask[j] != 0) {
      int h = a.hu[j];
      h = h < -1024 ? -1024 : (h > 3071 ? 3071 : h);
      rho = a.lut64[2 * (h + 1024)];
    }
    const long long mq = (long long)rint(rho * 4294967296.0);
    if (mq <= 0) continue;  // no mass: vacuum
    const unsigned long long t = (unsigned long long)a.tally[j];
    const Deposit d = {t >> 32, t & 0xFFFFFFFFull, (unsigned long long)mq};
    const unsigned row = j / (unsigned)a.nx;
    const int ix = (int)(j - row * (unsigned)a.nx), iy = (int)(row % (unsigned)a.ny), iz = (int)(row / (unsigned)a.ny);
    map_subvoxels<ALIGNED, B>(g, a.org, a.sp, n, ix, iy, iz, off, zf, zp, zb, tid,
                           [&](double qx, double qy, double qz) {
                             int tv[3];
                             if (ref_voxel(a, qx, qy, qz, tv)) count(a, win, d, tv);
                           });
    flush(a, win, d);
  }
}

// Source dose at q (mm): trilinear interpolation between voxel centres
// (x, then y, then z), the voxel-centre coordinate (q - origin) / spacing -
// 1/2 clamped to [0, n - 1] per axis; on the last plane both corners are the
// last voxel.
__device__ __forceinline__ double dose_sample(const DimPull &a, double qx, double qy, double qz) {
  const double q[3] = {qx, qy, qz};
  const int dims[3] = {a.snx, a.sny, a.snz};
  int lo[3], hi[3];
  double f[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double u = (q[k] - a.sorg[k]) / a.ssp[k] - 0.5;
    u = fmin(fmax(u, 0.0), (double)(dims[k] - 1));
    const int i = (int)floor(u);
    lo[k] = i;
    hi[k] = i + 1 < dims[k] ? i + 1 : dims[k] - 1;
    f[k] = u - (double)i;
  }
  const long long nx = a.snx, nxy = (long long)a.snx * a.sny;
  const double *d = a.sdose;
  const long long z0 = lo[2] * nxy, z1 = hi[2] * nxy, y0 = lo[1] * nx, y1 = hi[1] * nx;
  const double d000 = d[z0 + y0 + lo[0]], d100 = d[z0 + y0 + hi[0]];
  const double d010 = d[z0 + y1 + lo[0]], d110 = d[z0 + y1 + hi[0]];
  const double d001 = d[z1 + y0 + lo[0]], d101 = d[z1 + y0 + hi[0]];
  const double d011 = d[z1 + y1 + lo[0]], d111 = d[z1 + y1 + hi[0]];
  const double c00 = d000 + f[0] * (d100 - d000);
  const double c10 = d010 + f[0] * (d110 - d010);
  const double c01 = d001 + f[0] * (d101 - d001);
  const double c11 = d011 + f[0] * (d111 - d011);
  const double c0 = c00 + f[1] * (c10 - c00);
  const double c1 = c01 + f[1] * (c11 - c01);
  return c0 + f[2] * (c1 - c0);
}

template <bool ALIGNED, int B>
__global__ void __launch_bounds__(B) dim_pull(DimPull a) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double off[kMaxSub];
  const int n = a.n_sub;
  const int tid = threadIdx.x;
  double *zf = reinterpret_cast<double *>(smem);
  double *zp = zf + (size_t)n * B;
  int *zb = reinterpret_cast<int *>(zp + (size_t)n * B);
  if (tid < n) off[tid] = ((double)tid + 0.5) / (double)n;
  __syncthreads();
  const double count = (double)(n * n * n);
  const unsigned nvox = (unsigned)a.nx * (unsigned)a.ny * (unsigned)a.nz;
  const unsigned stride = gridDim.x * B;
  for (unsigned j = blockIdx.x * B + tid; j < nvox; j += stride) {
    const unsigned row = j / (unsigned)a.nx;
    const int ix = (int)(j - row * (unsigned)a.nx), iy = (int)(row % (unsigned)a.ny), iz = (int)(row / (unsigned)a.ny);
    // Eq. (3): the subvoxel samples summed in order (a centre outside the DVF
    // grid adds nothing), then divided by n^3
    double acc = 0.0;
    map_subvoxels<ALIGNED, B>(a.dvf, a.org, a.sp, n, ix, iy, iz, off, zf, zp, zb, tid,
                           [&](double qx, double qy, double qz) { acc = acc + dose_sample(a, qx, qy, qz); });
    a.dose[j] = a.dose[j] + acc / count;
  }
}

__global__ void __launch_bounds__(256) dvf_points_kernel(DvfDev d, double *x0, double *rf) {
  const long long np = (long long)d.n[0] * d.n[1] * d.n[2];
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += stride) {
    const double i = (double)(p % d.n[0]), j = (double)((p / d.n[0]) % d.n[1]),
                 k = (double)(p / ((long long)d.n[0] * d.n[1]));
    double x[3], m[3], r[3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
      x[a] = (d.u[a] * d.sp[0]) * i + (d.v[a] * d.sp[1]) * j + (d.w[a] * d.sp[2]) * k + d.start[a];
    m[0] = x[0];
    m[1] = x[1];
    m[2] = x[2];
    if (d.has_pre) rigid(d.pre, x, m);
#pragma unroll
    for (int a = 0; a < 3; ++a) r[a] = m[a] + d.delta[3 * p + a];
    if (d.has_post) {
      const double t[3] = {r[0], r[1], r[2]};
      rigid(d.post, t, r);
    }
    if (x0) {
#pragma unroll
      for (int a = 0; a < 3; ++a) x0[3 * p + a] = x[a];
    }
    if (rf) {
#pragma unroll
      for (int a = 0; a < 3; ++a) rf[3 * p + a] = r[a];
    }
  }
}

__global__ void __launch_bounds__(256) emtm_ratio(EmtmRatio a) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < a.nvox; i += stride) {
    const long long m = (long long)a.mass[i];
    if (m <= 0) continue;
    const double e = (double)a.e_hi[i] * 4294967296.0 + (double)a.e_lo[i];
    a.dose[i] = a.dose[i] + (e * 1.602176634e-13) / ((double)m * a.vol_cm3 * 1e-3 * a.n_hist);
  }
}

__global__ void __launch_bounds__(256) emtm_mask(EmtmMask a) {
  const long long nvox = (long long)a.nx * a.ny * a.nz;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nvox; i += stride) {
    const int ix = (int)(i % a.nx), iy = (int)((i / a.nx) % a.ny), iz = (int)(i / ((long long)a.nx * a.ny));
    const double cx = a.org[0] + ((double)ix + 0.5) * a.sp[0];
    const double cy = a.org[1] + ((double)iy + 0.5) * a.sp[1];
    const double cz = a.org[2] + ((double)iz + 0.5) * a.sp[2];
    bool in = true;
    for (int k = 0; k < a.n_dvf && in; ++k) {
      double g[3];
      in = dvf_coords(a.dvfs[k], cx, cy, cz, g);
    }
    if (!in) a.dose[i] = 0.0;
    if (a.mask_out && (a.first || !in)) a.mask_out[i] = in ? 1 : 0;
  }
}

unsigned grid_for(long long n, int block = 256) {
  long long b = (n + block - 1) / block;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

// Block size for a kernel whose threads each need `per_thread` bytes of LDS:
// 256, unless LDS (160 KiB per CU) then leaves fewer than 512 threads (two
// waves per SIMD) resident on a CU; then the one of 128 and 64 that keeps the
// most threads resident (measured: above two waves per SIMD smaller blocks
// gain nothing; below, n = 10 takes 280 instead of 425 ms).
int pick_block(size_t per_thread) {
  auto resident = [&](int b) -> long long {
    const size_t per_block = per_thread * (size_t)b;
    const long long blocks = per_block ? (long long)((160u * 1024u) / per_block) : 1280 / b;
    return std::min<long long>(blocks * b, 1280);
  };
  if (resident(256) >= 512) return 256;
  int best = 256;
  for (int b : {128, 64})
    if (resident(b) > resident(best)) best = b;
  return best;
}

template <bool ALIGNED, int B>
hipError_t launch_push_b(const EmtmPush &a, size_t per_thread, long long n, hipStream_t st) {
  const size_t lds = per_thread * B;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&emtm_push<ALIGNED, B>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((emtm_push<ALIGNED, B>), dim3(grid_for(n, B)), dim3(B), lds, st, a);
  return hipGetLastError();
}

template <bool ALIGNED>
hipError_t launch_push_a(const EmtmPush &a, size_t per_thread, long long n, hipStream_t st) {
  switch (pick_block(per_thread)) {
    case 64: return launch_push_b<ALIGNED, 64>(a, per_thread, n, st);
    case 128: return launch_push_b<ALIGNED, 128>(a, per_thread, n, st);
    default: return launch_push_b<ALIGNED, 256>(a, per_thread, n, st);
  }
}

template <bool ALIGNED, int B>
hipError_t launch_dim_b(const DimPull &a, size_t per_thread, long long n, hipStream_t st) {
  const size_t lds = per_thread * B;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&dim_pull<ALIGNED, B>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((dim_pull<ALIGNED, B>), dim3(grid_for(n, B)), dim3(B), lds, st, a);
  return hipGetLastError();
}

template <bool ALIGNED>
hipError_t launch_dim_a(const DimPull &a, size_t per_thread, long long n, hipStream_t st) {
  switch (pick_block(per_thread)) {
    case 64: return launch_dim_b<ALIGNED, 64>(a, per_thread, n, st);
    case 128: return launch_dim_b<ALIGNED, 128>(a, per_thread, n, st);
    default: return launch_dim_b<ALIGNED, 256>(a, per_thread, n, st);
  }
}

}  // namespace

hipError_t launch_emtm_push(const EmtmPush &a, hipStream_t st) {
  const long long n = (long long)a.nx * a.ny * a.nz;
  if (a.n_sub < 1 || a.n_sub > kMaxSub) return hipErrorInvalidValue;
  // per thread: the counting window, and the z table of the axis-aligned path
  const size_t per_thread = sizeof(uint32_t) * (kWinCells >> win_lg(a.n_sub)) +
                            (a.aligned ? (2 * sizeof(double) + sizeof(int)) * (size_t)a.n_sub : 0);
  return a.aligned ? launch_push_a<true>(a, per_thread, n, st) : launch_push_a<false>(a, per_thread, n, st);
}

hipError_t launch_dim_pull(const DimPull &a, hipStream_t st) {
  const long long n = (long long)a.nx * a.ny * a.nz;
  if (a.n_sub < 1 || a.n_sub > kMaxSub) return hipErrorInvalidValue;
  const size_t per_thread = a.aligned ? (2 * sizeof(double) + sizeof(int)) * (size_t)a.n_sub : 0;
  return a.aligned ? launch_dim_a<true>(a, per_thread, n, st) : launch_dim_a<false>(a, per_thread, n, st);
}

hipError_t launch_dvf_points(const DvfDev &d, double *x0, double *rf, hipStream_t st) {
  const long long n = (long long)d.n[0] * d.n[1] * d.n[2];
  hipLaunchKernelGGL(dvf_points_kernel, dim3(grid_for(n)), dim3(256), 0, st, d, x0, rf);
  return hipGetLastError();
}

hipError_t launch_emtm_ratio(const EmtmRatio &a, hipStream_t st) {
  hipLaunchKernelGGL(emtm_ratio, dim3(grid_for(a.nvox)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_emtm_mask(const EmtmMask &a, hipStream_t st) {
  const long long n = (long long)a.nx * a.ny * a.nz;
  hipLaunchKernelGGL(emtm_mask, dim3(grid_for(n)), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace pmc
