// Transport kernels of libpmc for gfx950.
//
//  transport_plain       one launch per phase, one history per thread, no refill
//  transport_persistent  one launch for all phases of a request: waves pop work
//                        items (spot, history range) from a global cursor and
//                        refill lanes whose proton has ended (ballot + rank)
//  trace_kernel          one history with a record per step (validation)
//  convert_kernel        int64 tally -> dose (Gy per history) and density
//  fill_u64_kernel       zero-fill used instead of memset inside captured graphs
//
// All transport kernels run the same `pmc::step`, so for equal inputs they
// produce bit-identical integer tallies whatever the schedule.
#include "pmc_device.hpp"
#include "pmc_internal.hpp"

namespace pmc {

// ---------------------------------------------------------------------------
// counters: per-lane totals -> block sums -> 128-bit global atomics
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long wave_sum(unsigned long long x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

__device__ __forceinline__ void add128(unsigned long long *p, unsigned long long lo,
                                       unsigned long long hi) {
  const unsigned long long old = __hip_atomic_fetch_add(p, lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (old + lo < old) hi += 1ull;
  if (hi) __hip_atomic_fetch_add(p + 1, hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Every thread of the block must call this (it synchronises the block).
// `red` is LDS of kNc * (waves + 1) words.
constexpr int kNc = 13;  // 3 energies as (lo32, hi32) sums + 7 event counts

__device__ void commit_counters(const LaneCounters &C, unsigned long long *counters,
                                unsigned long long *red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  unsigned long long v[kNc];
  v[0] = C.esc & 0xffffffffull; v[1] = C.esc >> 32;
  v[2] = C.nuc & 0xffffffffull; v[3] = C.nuc >> 32;
  v[4] = C.cut & 0xffffffffull; v[5] = C.cut >> 32;
  v[6] = C.hist; v[7] = C.steps; v[8] = C.delta; v[9] = C.nuc_ev; v[10] = C.escapes;
  v[11] = C.misses; v[12] = C.atomics;
#pragma unroll
  for (int k = 0; k < kNc; ++k) v[k] = wave_sum(v[k]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < kNc; ++k) red[wave * kNc + k] = v[k];
  }
  __syncthreads();
  unsigned long long *tot = red + kNc * nw;
  if (threadIdx.x < kNc) {
    unsigned long long s = 0;
    for (int w = 0; w < nw; ++w) s += red[w * kNc + threadIdx.x];
    tot[threadIdx.x] = s;
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < 3) {
    // energy e: value = hi32sum * 2^32 + lo32sum, as a 128-bit (lo, hi) pair
    const unsigned long long lo32 = tot[2 * t], hi32 = tot[2 * t + 1];
    const unsigned long long lo = lo32 + (hi32 << 32);
    const unsigned long long hi = (hi32 >> 32) + (lo < lo32 ? 1ull : 0ull);
    if (lo | hi) add128(counters + 2 * t, lo, hi);
  } else if (t >= 6 && t < kNc) {
    if (tot[t]) __hip_atomic_fetch_add(counters + kCHist + (t - 6), tot[t], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <typename R>
__device__ __forceinline__ Geo<R> geo_of(const TargetDev &t) {
  Geo<R> g;
  g.hu = t.hu;
  g.mask = t.mask;
  g.tally = t.tally;
  g.n[0] = t.nx; g.n[1] = t.ny; g.n[2] = t.nz;
  g.nxy = t.nx * t.ny;
  g.d[0] = (R)t.d[0]; g.d[1] = (R)t.d[1]; g.d[2] = (R)t.d[2];
  g.lut = t.lut;
  return g;
}

// LDS layout: [tables kNtab x R4][lut kLutSize x R2 (optional)][targets][reduction]
template <typename R> struct Smem {
  static constexpr size_t tab_bytes = sizeof(typename M<R>::R4) * kNtab;
  static constexpr size_t lut_bytes = sizeof(typename M<R>::R2) * kLutSize;
};

// ---------------------------------------------------------------------------
// plain engine: thread g -> g-th history of the phase's spot list
// ---------------------------------------------------------------------------
// FP64 (validation) kernels get more registers per lane
template <typename R> constexpr int kMaxBlock = sizeof(R) == 8 ? 256 : 1024;

template <typename R, bool LUT_LDS>
__global__ void __launch_bounds__(kMaxBlock<R>)
transport_plain(const SpotDev<R> *__restrict__ spots, const int32_t *__restrict__ spot_ids,
                const long long *__restrict__ first, int32_t n_list, long long n_hist,
                TargetDev target, const typename M<R>::R2 *__restrict__ lut_g,
                const typename M<R>::R4 *__restrict__ tab_g, R l2e0, R inv_dl2, R dl2,
                uint32_t k0, uint32_t k1, uint32_t flags, unsigned long long *counters) {
  extern __shared__ __align__(16) unsigned char smem[];
  using R2 = typename M<R>::R2;
  using R4 = typename M<R>::R4;
  R4 *tab_s = reinterpret_cast<R4 *>(smem);
  R2 *lut_s = reinterpret_cast<R2 *>(smem + Smem<R>::tab_bytes);
  unsigned long long *red = reinterpret_cast<unsigned long long *>(
      smem + Smem<R>::tab_bytes + (LUT_LDS ? Smem<R>::lut_bytes : 0));
  for (int i = threadIdx.x; i < kNtab; i += blockDim.x) tab_s[i] = tab_g[i];
  if constexpr (LUT_LDS)
    for (int i = threadIdx.x; i < kLutSize; i += blockDim.x) lut_s[i] = lut_g[i];
  __syncthreads();

  Tab<R> T;
  T.t = tab_s; T.l2e0 = l2e0; T.inv_dl2 = inv_dl2; T.dl2 = dl2;
  const R2 *lut = LUT_LDS ? lut_s : lut_g;
  const Geo<R> G = geo_of<R>(target);
  LaneCounters C = {};
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n_hist) {
    int lo = 0, hi = n_list;  // first[lo] <= g < first[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (first[mid] <= g) lo = mid; else hi = mid;
    }
    const int32_t s = spot_ids[lo];
    Lane<R> L;
    start_history(L, spots[s], s, (uint32_t)(g - first[lo]), G, k0, k1, C);
    while (L.fate == kAlive) step<R, false>(L, G, T, lut, k0, k1, flags, C, nullptr, 0);
    flush_tally(L, G, C);
  }
  commit_counters(C, counters, red);
}

// ---------------------------------------------------------------------------
// persistent engine: work queue + wave-level lane refill
// ---------------------------------------------------------------------------
template <typename R, bool LUT_LDS>
__global__ void __launch_bounds__(kMaxBlock<R>)
transport_persistent(const SpotDev<R> *__restrict__ spots, const WorkItem *__restrict__ items,
                     int32_t n_items, const TargetDev *__restrict__ targets, int32_t n_targets,
                     const typename M<R>::R2 *__restrict__ luts_g,
                     const typename M<R>::R4 *__restrict__ tab_g, R l2e0, R inv_dl2, R dl2,
                     uint32_t k0, uint32_t k1, uint32_t flags, int32_t refill_min,
                     unsigned long long *cursor, unsigned long long *counters) {
  extern __shared__ __align__(16) unsigned char smem[];
  using R2 = typename M<R>::R2;
  using R4 = typename M<R>::R4;
  R4 *tab_s = reinterpret_cast<R4 *>(smem);
  R2 *lut_s = reinterpret_cast<R2 *>(smem + Smem<R>::tab_bytes);
  // per-target geometry in the working precision, converted once per block
  Geo<R> *geo_s = reinterpret_cast<Geo<R> *>(smem + Smem<R>::tab_bytes +
                                             (LUT_LDS ? Smem<R>::lut_bytes : 0));
  unsigned long long *red = reinterpret_cast<unsigned long long *>(geo_s + n_targets);
  for (int i = threadIdx.x; i < kNtab; i += blockDim.x) tab_s[i] = tab_g[i];
  if constexpr (LUT_LDS)
    for (int i = threadIdx.x; i < kLutSize; i += blockDim.x) lut_s[i] = luts_g[i];
  for (int i = threadIdx.x; i < n_targets; i += blockDim.x) geo_s[i] = geo_of<R>(targets[i]);
  __syncthreads();

  Tab<R> T;
  T.t = tab_s; T.l2e0 = l2e0; T.inv_dl2 = inv_dl2; T.dl2 = dl2;
  const int lane = threadIdx.x & 63;
  LaneCounters C = {};
  Lane<R> L;
  L.fate = kMissed;  // idle
  int32_t tgt = 0;
  // wave-uniform state of the work item being drained
  int32_t it_spot = 0;
  uint32_t it_next = 0, it_end = 0;
  bool drained = false;

  for (;;) {
    unsigned long long idle = __ballot(L.fate != kAlive);
    if (!drained && (int)__popcll(idle) >= refill_min) {
      while (idle != 0ull) {
        if (it_next == it_end) {
          unsigned long long k = 0;
          if (lane == 0) k = __hip_atomic_fetch_add(cursor, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          k = __shfl(k, 0, 64);
          if (k >= (unsigned long long)n_items) { drained = true; break; }
          const WorkItem wi = items[k];
          it_spot = __builtin_amdgcn_readfirstlane(wi.spot);
          it_next = __builtin_amdgcn_readfirstlane(wi.h_begin);
          it_end = it_next + __builtin_amdgcn_readfirstlane(wi.h_count);
        }
        const uint32_t n_idle = (uint32_t)__popcll(idle);
        const uint32_t avail = it_end - it_next;
        const uint32_t take = avail < n_idle ? avail : n_idle;
        const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(idle >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)idle, 0u));
        const bool me_idle = (idle >> lane) & 1ull;
        const bool mine = me_idle && rank < take;
        if (mine) {
          const SpotDev<R> &sp = spots[it_spot];
          tgt = sp.target;
          start_history(L, sp, it_spot, it_next + rank, geo_s[tgt], k0, k1, C);
        }
        it_next += take;
        idle = __ballot(me_idle && !mine);
      }
    }
    const bool alive = L.fate == kAlive;
    if (!__any(alive)) {
      if (drained) break;
      continue;
    }
    if (alive) {
      const Geo<R> G = geo_s[tgt];
      const R2 *lut = LUT_LDS ? lut_s : luts_g + (size_t)G.lut * kLutSize;
      step<R, false>(L, G, T, lut, k0, k1, flags, C, nullptr, 0);
      if (L.fate != kAlive) flush_tally(L, G, C);
    }
  }
  commit_counters(C, counters, red);
}

// ---------------------------------------------------------------------------
// trace of a single history (validation; tables and LUT in global memory)
// ---------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(64) trace_kernel(SpotDev<R> sp, int32_t spot, uint32_t h, TargetDev target,
                             const typename M<R>::R2 *lut_g, const typename M<R>::R4 *tab_g,
                             R l2e0, R inv_dl2, R dl2, uint32_t k0, uint32_t k1, uint32_t flags,
                             TraceRec *rec, int32_t max_rec, int32_t *n_rec) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  Tab<R> T;
  T.t = tab_g; T.l2e0 = l2e0; T.inv_dl2 = inv_dl2; T.dl2 = dl2;
  const Geo<R> G = geo_of<R>(target);
  LaneCounters C = {};
  Lane<R> L;
  start_history(L, sp, spot, h, G, k0, k1, C);
  L.nsteps = 0;
  trace_out(rec, 0, max_rec, -1, L.v, L, G, (R)0, 0ll, (R)0);
  while (L.fate == kAlive) step<R, true>(L, G, T, lut_g, k0, k1, flags, C, rec, max_rec);
  flush_tally(L, G, C);
  *n_rec = (int32_t)L.nsteps + 1;
}

// ---------------------------------------------------------------------------
// dose conversion: D = (t 2^-32 MeV->J) / (rho V 1e-3 kg) / N
// ---------------------------------------------------------------------------
__global__ void convert_kernel(const long long *__restrict__ tally, const int16_t *__restrict__ hu,
                               const uint8_t *__restrict__ mask, const double2 *__restrict__ lut64,
                               long long nvox, double vol_cm3, double n_hist,
                               double *__restrict__ dose, double *__restrict__ density) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < nvox; v += stride) {
    double rho = lut64[clamp_hu<double>(hu[v])].x;
    if (mask && mask[v] == 0) rho = 0.0;
    if (density) density[v] = rho;
    if (dose) {
      if (rho > 0.0) {
        const double e_j = (double)tally[v] / 4294967296.0 * 1.602176634e-13;
        const double m_kg = rho * vol_cm3 * 1e-3;
        dose[v] = e_j / m_kg / n_hist;
      } else {
        dose[v] = 0.0;
      }
    }
  }
}

__global__ void fill_u64_kernel(unsigned long long *p, long long n, unsigned long long value) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = value;
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
template <typename R>
static hipError_t launch_plain_t(const PlainLaunch &a, hipStream_t st) {
  using R2 = typename M<R>::R2;
  using R4 = typename M<R>::R4;
  const size_t red_bytes = sizeof(unsigned long long) * kNc * (a.block / 64 + 1);
  const size_t lds = Smem<R>::tab_bytes + (a.lut_lds ? Smem<R>::lut_bytes : 0) + red_bytes;
  const long long nb = (a.n_hist + a.block - 1) / a.block;
  if (nb <= 0) return hipSuccess;
  if (a.lut_lds)
    hipLaunchKernelGGL((transport_plain<R, true>), dim3((unsigned)nb), dim3(a.block), lds, st,
                       (const SpotDev<R> *)a.spots, a.spot_ids, a.first, a.n_list, a.n_hist,
                       a.target, (const R2 *)a.lut, (const R4 *)a.tab, (R)a.l2e0, (R)a.inv_dl2,
                       (R)a.dl2, a.k0, a.k1, a.flags, a.counters);
  else
    hipLaunchKernelGGL((transport_plain<R, false>), dim3((unsigned)nb), dim3(a.block), lds, st,
                       (const SpotDev<R> *)a.spots, a.spot_ids, a.first, a.n_list, a.n_hist,
                       a.target, (const R2 *)a.lut, (const R4 *)a.tab, (R)a.l2e0, (R)a.inv_dl2,
                       (R)a.dl2, a.k0, a.k1, a.flags, a.counters);
  return hipGetLastError();
}

template <typename R>
static hipError_t launch_persistent_t(const PersistentLaunch &a, hipStream_t st) {
  using R2 = typename M<R>::R2;
  using R4 = typename M<R>::R4;
  const size_t lds = persistent_lds<R>(a);
  if (a.lut_lds)
    hipLaunchKernelGGL((transport_persistent<R, true>), dim3(a.grid), dim3(a.block), lds, st,
                       (const SpotDev<R> *)a.spots, a.items, a.n_items, a.targets, a.n_targets,
                       (const R2 *)a.luts, (const R4 *)a.tab, (R)a.l2e0, (R)a.inv_dl2, (R)a.dl2,
                       a.k0, a.k1, a.flags, a.refill_min, a.cursor, a.counters);
  else
    hipLaunchKernelGGL((transport_persistent<R, false>), dim3(a.grid), dim3(a.block), lds, st,
                       (const SpotDev<R> *)a.spots, a.items, a.n_items, a.targets, a.n_targets,
                       (const R2 *)a.luts, (const R4 *)a.tab, (R)a.l2e0, (R)a.inv_dl2, (R)a.dl2,
                       a.k0, a.k1, a.flags, a.refill_min, a.cursor, a.counters);
  return hipGetLastError();
}

template <typename R>
static size_t persistent_lds(const PersistentLaunch &a) {
  return Smem<R>::tab_bytes + (a.lut_lds ? Smem<R>::lut_bytes : 0) +
         sizeof(Geo<R>) * (size_t)a.n_targets + sizeof(unsigned long long) * kNc * (a.block / 64 + 1);
}

template <typename R>
static int blocks_per_cu_t(const PersistentLaunch &a) {
  int n = 0;
  hipError_t e;
  if (a.lut_lds)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, transport_persistent<R, true>, a.block,
                                                     persistent_lds<R>(a));
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, transport_persistent<R, false>, a.block,
                                                     persistent_lds<R>(a));
  return e == hipSuccess ? n : 1;
}

int persistent_blocks_per_cu(const PersistentLaunch &a, bool fp64) {
  return fp64 ? blocks_per_cu_t<double>(a) : blocks_per_cu_t<float>(a);
}

hipError_t launch_plain(const PlainLaunch &a, bool fp64, hipStream_t st) {
  return fp64 ? launch_plain_t<double>(a, st) : launch_plain_t<float>(a, st);
}

hipError_t launch_persistent(const PersistentLaunch &a, bool fp64, hipStream_t st) {
  return fp64 ? launch_persistent_t<double>(a, st) : launch_persistent_t<float>(a, st);
}

hipError_t launch_trace(const TraceLaunch &a, bool fp64, hipStream_t st) {
  if (fp64) {
    hipLaunchKernelGGL(trace_kernel<double>, dim3(1), dim3(64), 0, st,
                       *(const SpotDev<double> *)a.spot, a.spot_index, a.h, a.target,
                       (const double2 *)a.lut, (const double4 *)a.tab, a.l2e0, a.inv_dl2, a.dl2,
                       a.k0, a.k1, a.flags, (TraceRec *)a.rec, a.max_rec, a.n_rec);
  } else {
    hipLaunchKernelGGL(trace_kernel<float>, dim3(1), dim3(64), 0, st,
                       *(const SpotDev<float> *)a.spot, a.spot_index, a.h, a.target,
                       (const float2 *)a.lut, (const float4 *)a.tab, (float)a.l2e0,
                       (float)a.inv_dl2, (float)a.dl2, a.k0, a.k1, a.flags, (TraceRec *)a.rec,
                       a.max_rec, a.n_rec);
  }
  return hipGetLastError();
}

hipError_t launch_convert(const long long *tally, const int16_t *hu, const uint8_t *mask,
                          const void *lut64, long long nvox, double vol_cm3, double n_hist,
                          double *dose, double *density, hipStream_t st) {
  const int block = 256;
  long long nb = (nvox + block - 1) / block;
  if (nb > 8192) nb = 8192;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(convert_kernel, dim3((unsigned)nb), dim3(block), 0, st, tally, hu, mask,
                     (const double2 *)lut64, nvox, vol_cm3, n_hist, dose, density);
  return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, long long n, unsigned long long value,
                           hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int block = 256;
  long long nb = (n + block - 1) / block;
  if (nb > 8192) nb = 8192;
  hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)nb), dim3(block), 0, st, p, n, value);
  return hipGetLastError();
}

}  // namespace pmc
