// Deformable dose accumulation by energy/mass transfer (Sec. 2.D.2, Eqs. (2),
// (4)-(6)) with DVFs stored as in App. B (Eqs. (7)-(8)).
//
//  emtm_push    one thread per source voxel: its n^3 subvoxel centres are
//               mapped to the reference grid (trilinear interpolation of the
//               DVF translations, FP64); the voxel's energy (tally, as two
//               32-bit halves) and mass units (round(rho 2^32)) are added,
//               once per subvoxel, to the reference voxel each centre lands
//               in.  A thread merges its subvoxels by target (up to 8 targets
//               in registers) before its atomics: a voxel usually maps into
//               few reference voxels.
//  emtm_ratio   dose_i += sum E / sum M (Eq. (5)) per reference voxel, in
//               Gy per history, added in source order (Eq. (2)).
//  emtm_mask    keeps the dose where the reference voxel centre lies in the
//               grid box of every DVF.
//
// Every floating-point decision (which reference voxel a centre lands in)
// uses the same FP64 operations in the same order as a plain evaluation of
// the formulas (no contraction), and every sum is an integer sum, so the
// result does not depend on the schedule.
#include <hip/hip_runtime.h>

#include "pmc_internal.hpp"

namespace pmc {

namespace {

constexpr int kTargets = 8;

__device__ __forceinline__ bool dvf_coords(const DvfDev &d, double px, double py, double pz, double g[3]) {
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

// T(r) of Eq. (1): r plus the trilinear interpolation (x, then y, then z) of
// the translations of the 8 grid points around r.  False outside the grid.
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
    q[k] = p[k] + (c0 + f[2] * (c1 - c0));
  }
  return true;
}

__device__ __forceinline__ void add_u64(unsigned long long *p, unsigned long long v) {
  __hip_atomic_fetch_add((__attribute__((address_space(1))) unsigned long long *)p, v, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void __launch_bounds__(256) emtm_push(EmtmPush a) {
  const long long nvox = (long long)a.nx * a.ny * a.nz;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x; j < nvox; j += stride) {
    double rho = 0.0;
    if (!a.mask || a.mask[j] != 0) {
      int h = a.hu[j];
      h = h < -1024 ? -1024 : (h > 3071 ? 3071 : h);
      rho = a.lut64[2 * (h + 1024)];
    }
    const long long mq = (long long)rint(rho * 4294967296.0);
    if (mq <= 0) continue;  // no mass: vacuum
    const unsigned long long t = (unsigned long long)a.tally[j];
    const unsigned long long t_hi = t >> 32, t_lo = t & 0xFFFFFFFFull;
    const int ix = (int)(j % a.nx), iy = (int)((j / a.nx) % a.ny), iz = (int)(j / ((long long)a.nx * a.ny));
    int tgt[kTargets], cnt[kTargets];
    int used = 0;
    auto flush = [&]() {
      for (int e = 0; e < used; ++e) {
        const unsigned long long c = (unsigned long long)cnt[e];
        if (t_hi) add_u64(a.e_hi + tgt[e], c * t_hi);
        if (t_lo) add_u64(a.e_lo + tgt[e], c * t_lo);
        add_u64(a.mass + tgt[e], c * (unsigned long long)mq);
      }
      used = 0;
    };
    const double n = (double)a.n_sub;
    for (int sc = 0; sc < a.n_sub; ++sc) {
      for (int sb = 0; sb < a.n_sub; ++sb) {
        for (int sa = 0; sa < a.n_sub; ++sa) {
          // subvoxel centre: origin + (index + (s + 0.5) / n) spacing
          const double px = a.org[0] + ((double)ix + ((double)sa + 0.5) / n) * a.sp[0];
          const double py = a.org[1] + ((double)iy + ((double)sb + 0.5) / n) * a.sp[1];
          const double pz = a.org[2] + ((double)iz + ((double)sc + 0.5) / n) * a.sp[2];
          double q[3];
          if (!dvf_map(a.dvf, px, py, pz, q)) continue;
          const double fx = floor((q[0] - a.rorg[0]) / a.rsp[0]);
          const double fy = floor((q[1] - a.rorg[1]) / a.rsp[1]);
          const double fz = floor((q[2] - a.rorg[2]) / a.rsp[2]);
          if (!(fx >= 0.0 && fx < (double)a.rnx && fy >= 0.0 && fy < (double)a.rny && fz >= 0.0 &&
                fz < (double)a.rnz))
            continue;
          const int i = (int)fx + a.rnx * ((int)fy + a.rny * (int)fz);
          int e = 0;
          while (e < used && tgt[e] != i) ++e;
          if (e < used) {
            cnt[e] += 1;
          } else {
            if (used == kTargets) flush();
            tgt[used] = i;
            cnt[used] = 1;
            ++used;
          }
        }
      }
    }
    flush();
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

unsigned grid_for(long long n) {
  long long b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

hipError_t launch_emtm_push(const EmtmPush &a, hipStream_t st) {
  const long long n = (long long)a.nx * a.ny * a.nz;
  hipLaunchKernelGGL(emtm_push, dim3(grid_for(n)), dim3(256), 0, st, a);
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
