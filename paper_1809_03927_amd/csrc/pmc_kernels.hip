// Transport kernels of libpmc for gfx950.
//
//  transport_plain       one launch per phase, one history per thread, no refill
//  transport_persistent  one launch for all phases of a request: waves pop work
//                        items (spot, history range) from a global cursor and
//                        refill lanes whose proton has ended (ballot + rank)
//  trace_kernel          one history with a record per step (validation)
//  convert_kernel        int64 tally -> dose (Gy per history) and density
//  fill_u64_kernel       zero-fill used instead of memset inside captured graphs
//  influence_*           per-spot box tallies -> thresholded CSR rows
//
// All transport kernels run the same `pmc::step`, so for equal inputs they
// produce bit-identical integer tallies whatever the schedule.
#include <mutex>

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
constexpr int kNc = 15;  // 4 energies as (lo32, hi32) sums + 7 event counts

__device__ void commit_counters(const LaneCounters &C, unsigned long long *counters,
                                unsigned long long *red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  unsigned long long v[kNc];
  v[0] = C.esc & 0xffffffffull; v[1] = C.esc >> 32;
  v[2] = C.nuc & 0xffffffffull; v[3] = C.nuc >> 32;
  v[4] = C.cut & 0xffffffffull; v[5] = C.cut >> 32;
  v[6] = C.hist; v[7] = C.steps; v[8] = C.delta; v[9] = C.nuc_ev; v[10] = C.escapes;
  v[11] = C.misses; v[12] = C.atomics;
  v[13] = C.out & 0xffffffffull; v[14] = C.out >> 32;
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
  if (t < 4) {
    // energy e: value = hi32sum * 2^32 + lo32sum, as a 128-bit (lo, hi) pair;
    // escaped, nuclear, cutoff at words 0-5, outside-box at words 13-14
    const int src = t < 3 ? 2 * t : 13;
    const unsigned long long lo32 = tot[src], hi32 = tot[src + 1];
    const unsigned long long lo = lo32 + (hi32 << 32);
    const unsigned long long hi = (hi32 >> 32) + (lo < lo32 ? 1ull : 0ull);
    if (lo | hi) add128(counters + src, lo, hi);
  } else if (t >= 6 && t < 13) {
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
template <typename R, bool LUT_LDS, bool BOX>
__global__ void __launch_bounds__(kMaxBlock<R>)
transport_persistent(const SpotDev<R> *__restrict__ spots, const WorkItem *__restrict__ items,
                     int32_t n_items, const TargetDev *__restrict__ targets, int32_t n_targets,
                     const typename M<R>::R2 *__restrict__ luts_g,
                     const typename M<R>::R4 *__restrict__ tab_g, R l2e0, R inv_dl2, R dl2,
                     uint32_t k0, uint32_t k1, uint32_t flags, int32_t refill_min,
                     unsigned long long *cursor, unsigned long long *counters,
                     const BoxDev *__restrict__ boxes, unsigned long long *box_tally,
                     long long box_bias, unsigned int *drained_flag) {
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
  BoxLane B = {};
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
          if (k >= (unsigned long long)n_items) {
            drained = true;
            // every work item is taken: tell the host (pinned memory, vector
            // store) so that it can start the next launch during this drain
            if (drained_flag && lane == 0)
              __hip_atomic_store(drained_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            break;
          }
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
          if constexpr (BOX) {
            const BoxDev &bx = boxes[it_spot];
            B.base = box_tally + (bx.offset - box_bias);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
              B.lo[k] = bx.lo[k];
              B.n[k] = bx.n[k];
            }
          }
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
      constexpr int TM = BOX ? kTallyBox : kTallyGrid;
      step<R, false, TM>(L, G, T, lut, k0, k1, flags, C, nullptr, 0, B);
      if (L.fate != kAlive) flush_tally<R, TM>(L, G, C, B);
    }
  }
  commit_counters(C, counters, red);
}

// ---------------------------------------------------------------------------
// block engine: a block runs one work item (a run of one spot's histories)
// at a time with all of its waves.  Deposits inside the spot's core box add
// into the block's LDS copy of the core, the others into the phase tally;
// when every history of the item has ended, the block adds each nonzero core
// entry into the tally: one global atomic per voxel instead of one per voxel
// visit.  Waves refill idle lanes from the item through an LDS counter.
// With BOX (influence calculations) the lanes tally into their spot's box as
// in transport_persistent, and the core is a window of that box whose entries
// are flushed into the box tally.
// ---------------------------------------------------------------------------
size_t core_fixed_lds(bool lut_lds) {
  return Smem<float>::tab_bytes + (lut_lds ? Smem<float>::lut_bytes : 0) +
         sizeof(unsigned long long) * kNc * (kCoreBlock / 64 + 1) + 16;
}

template <typename R, bool LUT_LDS, bool BOX, bool LOG = false, bool SLICE = false>
__global__ void __launch_bounds__(kCoreBlock)
transport_core(const SpotDev<R> *__restrict__ spots, const WorkItem *__restrict__ items,
               int32_t n_items, const TargetDev *__restrict__ targets,
               const typename M<R>::R2 *__restrict__ luts_g,
               const typename M<R>::R4 *__restrict__ tab_g, R l2e0, R inv_dl2, R dl2,
               uint32_t k0, uint32_t k1, uint32_t flags, int32_t refill_min,
               unsigned long long *cursor, unsigned long long *counters,
               const SliceCore *__restrict__ slices, const CoreDev *__restrict__ cores, int32_t core_cap,
               const BoxDev *__restrict__ boxes,
               unsigned long long *box_tally, long long box_bias, unsigned int *drained_flag,
               unsigned long long *log, uint32_t log_cap, uint32_t *log_count) {
  static_assert(!(LOG && BOX), "the address log covers the phase tallies");
  constexpr int TM = BOX ? (SLICE ? kTallyBoxSlice : kTallyBoxCore)
                         : (SLICE ? (LOG ? kTallySliceLog : kTallySlice) : (LOG ? kTallyCoreLog : kTallyCore));
  extern __shared__ __align__(16) unsigned char smem[];
  using R2 = typename M<R>::R2;
  using R4 = typename M<R>::R4;
  // LDS layout: [tables][lut (optional)][reduction][item state][core tally]
  R4 *tab_s = reinterpret_cast<R4 *>(smem);
  R2 *lut_s = reinterpret_cast<R2 *>(smem + Smem<R>::tab_bytes);
  unsigned long long *red = reinterpret_cast<unsigned long long *>(
      smem + Smem<R>::tab_bytes + (LUT_LDS ? Smem<R>::lut_bytes : 0));
  int32_t *state = reinterpret_cast<int32_t *>(red + kNc * (kCoreBlock / 64 + 1));  // item, next
  unsigned long long *core = reinterpret_cast<unsigned long long *>(state + 4);
  for (int i = threadIdx.x; i < kNtab; i += blockDim.x) tab_s[i] = tab_g[i];
  if constexpr (LUT_LDS)
    for (int i = threadIdx.x; i < kLutSize; i += blockDim.x) lut_s[i] = luts_g[i];
  for (int i = threadIdx.x; i < core_cap; i += blockDim.x) core[i] = 0ull;

  Tab<R> T;
  T.t = tab_s; T.l2e0 = l2e0; T.inv_dl2 = inv_dl2; T.dl2 = dl2;
  const int lane = threadIdx.x & 63;
  LaneCounters C = {};
  Lane<R> L;
  L.fate = kMissed;  // idle
  for (;;) {
    if (threadIdx.x == 0) {
      const unsigned long long k = __hip_atomic_fetch_add(cursor, 1ull, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT);
      state[0] = k < (unsigned long long)n_items ? (int32_t)k : -1;
      state[1] = 0;
      // every work item is taken: tell the host (pinned memory, vector store)
      if (k >= (unsigned long long)n_items && drained_flag)
        __hip_atomic_store(drained_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    // the item is published; tables, the zeroed core and the previous flush are complete
    __syncthreads();
    const int32_t k = __builtin_amdgcn_readfirstlane(state[0]);
    if (k < 0) break;
    const int32_t spot = __builtin_amdgcn_readfirstlane(items[k].spot);
    const uint32_t h_begin = __builtin_amdgcn_readfirstlane(items[k].h_begin);
    const uint32_t count = __builtin_amdgcn_readfirstlane(items[k].h_count);
    const SpotDev<R> &sp = spots[spot];
    const int32_t tgt = __builtin_amdgcn_readfirstlane(sp.target);
    const Geo<R> G = geo_of<R>(targets[tgt]);
    const R2 *lut = LUT_LDS ? lut_s : luts_g + (size_t)G.lut * kLutSize;
    // the spot's core: a window of its box (influence calculations with
    // straight cores) or its slices
    int32_t cn[3] = {0, 0, 0}, clo[3] = {0, 0, 0};
    long long n_core;
    BoxLane B;
    if constexpr (BOX && !SLICE) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        clo[a] = __builtin_amdgcn_readfirstlane(cores[spot].lo[a]);
        cn[a] = __builtin_amdgcn_readfirstlane(cores[spot].n[a]);
      }
      n_core = (long long)cn[0] * cn[1] * cn[2];
    } else {
      const SliceCore &sc = slices[spot];
      B.sd = __builtin_amdgcn_readfirstlane(sc.d);
      B.sa = B.sd == 2 ? 0 : B.sd + 1;
      B.se = B.sd == 0 ? 2 : B.sd - 1;
      B.sj0 = __builtin_amdgcn_readfirstlane(sc.j0);
      B.sn = __builtin_amdgcn_readfirstlane(sc.n_sl);
      B.swa = __builtin_amdgcn_readfirstlane(sc.wa);
      B.swe = __builtin_amdgcn_readfirstlane(sc.we);
      B.scells = B.swa * B.swe;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        B.sA[i] = __builtin_amdgcn_readfirstlane(sc.A[i]);
        B.sB[i] = __builtin_amdgcn_readfirstlane(sc.B[i]);
        B.smin[i] = __builtin_amdgcn_readfirstlane(sc.amin[i]);
        B.smax[i] = __builtin_amdgcn_readfirstlane(sc.amax[i]);
      }
      n_core = (long long)B.sn * B.scells;
      // without SLICE every core of the launch is straight (a beam along a
      // grid axis: constant corners), a box of the grid; one that is not is
      // left without a core
      if constexpr (!SLICE)
        if (B.sB[0] != 0 || B.sB[1] != 0) n_core = 0;
    }
    const bool use_core = n_core > 0 && n_core <= (long long)core_cap;
    if constexpr (BOX) {
      // the box's first entry relative to this batch's scratch (64-bit)
      const unsigned long long rel = (unsigned long long)(boxes[spot].offset - box_bias);
      const uint32_t rel_lo = __builtin_amdgcn_readfirstlane((uint32_t)rel);
      const uint32_t rel_hi = __builtin_amdgcn_readfirstlane((uint32_t)(rel >> 32));
      B.base = box_tally + (long long)(((unsigned long long)rel_hi << 32) | rel_lo);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        B.lo[a] = __builtin_amdgcn_readfirstlane(boxes[spot].lo[a]);
        B.n[a] = __builtin_amdgcn_readfirstlane(boxes[spot].n[a]);
        B.clo[a] = clo[a];
        B.cn[a] = use_core ? cn[a] : 0;  // no core: the box tally takes every deposit
      }
      if constexpr (SLICE)
        if (!use_core) B.sn = 0;
      B.core = core;
    } else {
      B.base = core;
      if (!use_core) B.sn = 0;  // no core: every deposit goes to the tally
      if constexpr (!SLICE) {
        // the straight core as a box of the grid, entries x fastest
        const int32_t c0 = slice_corner(B.sA[0], 0, 0, B.smin[0], B.smax[0]);
        const int32_t c1 = slice_corner(B.sA[1], 0, 0, B.smin[1], B.smax[1]);
        const int32_t sn = B.sn;
        B.lo[0] = B.sd == 0 ? B.sj0 : (B.sa == 0 ? c0 : c1);
        B.lo[1] = B.sd == 1 ? B.sj0 : (B.sa == 1 ? c0 : c1);
        B.lo[2] = B.sd == 2 ? B.sj0 : (B.sa == 2 ? c0 : c1);
        B.n[0] = B.sd == 0 ? sn : (B.sa == 0 ? B.swa : B.swe);
        B.n[1] = B.sd == 1 ? sn : (B.sa == 1 ? B.swa : B.swe);
        B.n[2] = B.sd == 2 ? sn : (B.sa == 2 ? B.swa : B.swe);
      }
      if constexpr (LOG) {
        B.log = log;
        B.log_cap = log_cap;
        B.log_stride = gridDim.x * blockDim.x;
        B.log_lane = blockIdx.x * blockDim.x + threadIdx.x;
      }
    }
    bool taken_all = false;
    for (;;) {
      const unsigned long long idle = __ballot(L.fate != kAlive);
      if (!taken_all && (int)__popcll(idle) >= refill_min) {
        const uint32_t n_idle = (uint32_t)__popcll(idle);
        uint32_t h0 = 0;
        if (lane == 0)
          h0 = __hip_atomic_fetch_add(reinterpret_cast<uint32_t *>(state + 1), n_idle, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_WORKGROUP);
        h0 = __shfl(h0, 0, 64);
        const uint32_t avail = h0 < count ? count - h0 : 0u;
        const uint32_t take = avail < n_idle ? avail : n_idle;
        if (h0 + n_idle >= count) taken_all = true;
        const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(idle >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)idle, 0u));
        const bool mine = ((idle >> lane) & 1ull) && rank < take;
        if (mine) start_history(L, sp, spot, h_begin + h0 + rank, G, k0, k1, C);
      }
      const bool alive = L.fate == kAlive;
      if (!__any(alive)) {
        if (taken_all) break;
        continue;
      }
      if (alive) {
        step<R, false, TM>(L, G, T, lut, k0, k1, flags, C, nullptr, 0, B);
        if (L.fate != kAlive) flush_tally<R, TM>(L, G, C, B);
      }
    }
    __syncthreads();  // every history of the item has ended: the core is complete
    if (use_core) {
      for (int e = threadIdx.x; e < (int)n_core; e += blockDim.x) {
        const unsigned long long v = core[e];
        if (v) {
          core[e] = 0ull;
          if constexpr (BOX && !SLICE) {
            const int32_t nxy = cn[0] * cn[1];
            const int32_t z = e / nxy, r = e - z * nxy, y = r / cn[0], x = r - y * cn[0];
            const int32_t bx = clo[0] - B.lo[0] + x, by = clo[1] - B.lo[1] + y, bz = clo[2] - B.lo[2] + z;
            atomic_add_u64(&B.base[bx + B.n[0] * (by + B.n[1] * bz)], v);
          } else if constexpr (!SLICE) {
            const int32_t nxy = B.n[0] * B.n[1];
            const int32_t z = e / nxy, r = e - z * nxy, y = r / B.n[0], x = r - y * B.n[0];
            const int32_t vox = (B.lo[0] + x) + G.n[0] * ((B.lo[1] + y) + G.n[1] * (B.lo[2] + z));
            atomic_add_u64(&G.tally[vox], v);
            if constexpr (LOG) log_atomic(B, C.atomics, &G.tally[vox]);
          } else {
            // entry -> slice j, across (x, y) -> grid voxel
            const int32_t j = e / B.scells, r = e - j * B.scells, y = r / B.swa, x = r - y * B.swa;
            const int32_t cd = B.sj0 + j;
            const int32_t ca = slice_corner(B.sA[0], B.sB[0], j, B.smin[0], B.smax[0]) + x;
            const int32_t ce = slice_corner(B.sA[1], B.sB[1], j, B.smin[1], B.smax[1]) + y;
            const int32_t ix = B.sd == 0 ? cd : (B.sa == 0 ? ca : ce);
            const int32_t iy = B.sd == 1 ? cd : (B.sa == 1 ? ca : ce);
            const int32_t iz = B.sd == 2 ? cd : (B.sa == 2 ? ca : ce);
            if constexpr (BOX) {  // the slices lie inside the box
              atomic_add_u64(&B.base[(ix - B.lo[0]) + B.n[0] * ((iy - B.lo[1]) + B.n[1] * (iz - B.lo[2]))], v);
            } else {
              const int32_t vox = ix + G.n[0] * (iy + G.n[1] * iz);
              atomic_add_u64(&G.tally[vox], v);
              if constexpr (LOG) log_atomic(B, C.atomics, &G.tally[vox]);
            }
          }
          C.atomics += 1;
        }
      }
    }
  }
  if constexpr (LOG) log_count[blockIdx.x * blockDim.x + threadIdx.x] = C.atomics;
  commit_counters(C, counters, red);
}

// ---------------------------------------------------------------------------
// replay of a logged deposit-address pattern: lane g issues its logged
// 64-bit atomics, in its order, back to back (one per loop iteration, value
// 1) -- the atomic throughput of exactly those addresses without the
// transport around them
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kCoreBlock) atomic_replay(const unsigned long long *__restrict__ log,
                                                             uint32_t log_cap,
                                                             const uint32_t *__restrict__ log_count,
                                                             uint32_t n_lanes) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_lanes) return;
  const uint32_t c = log_count[g];
  const uint32_t n = c < log_cap ? c : log_cap;
  for (uint32_t k = 0; k < n; ++k)
    atomic_add_u64(reinterpret_cast<unsigned long long *>(log[(size_t)k * n_lanes + g]), 1ull);
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
// influence matrix: per-spot box tallies -> CSR rows, in tiles of kTile box
// entries (no tile straddles two spots: box offsets are multiples of kTile).
// Thread i of a tile handles entries i, i + 256, i + 512, i + 768, so loads
// of the box tallies are coalesced and the entries of a wave are consecutive.
// ---------------------------------------------------------------------------
constexpr int kInfBlock = 256;
constexpr int kWriteTiles = 64;  // influence_write: consecutive tiles per block (one wave reads their counts)
static_assert(kTile == 4 * kInfBlock, "tile = 4 entries per thread");

__device__ __forceinline__ int tile_owner(const long long *tile_first, int n_spots, long long t) {
  int lo = 0, hi = n_spots;  // tile_first[lo] <= t < tile_first[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (tile_first[mid] <= t) lo = mid; else hi = mid;
  }
  return lo;
}

struct InfEntry {
  long long T;   // box tally, 2^-32 MeV
  double rho;    // density (0 outside the external mask); set only when T > 0
  int32_t v;     // voxel of the phase grid; set only when T > 0
};

// Box entry e (< 2^31: a box is never larger than its grid) of spot box bx,
// whose tally T is already loaded; the voxel and its density are looked up
// only for entries with energy (the ~90 % of empty entries cost nothing more).
__device__ __forceinline__ InfEntry inf_entry_of(const InfluenceLaunch &a, const BoxDev &bx, long long T,
                                                 int32_t e) {
  InfEntry r;
  r.T = T;
  r.rho = 0.0;
  r.v = 0;
  if (r.T > 0) {
    const uint32_t n0 = (uint32_t)bx.n[0], n1 = (uint32_t)bx.n[1];
    const uint32_t yz = (uint32_t)e / n0;
    const uint32_t x = (uint32_t)e - yz * n0;
    const uint32_t z = yz / n1;
    const uint32_t y = yz - z * n1;
    r.v = (bx.lo[0] + (int32_t)x) + a.nx * ((bx.lo[1] + (int32_t)y) + a.ny * (bx.lo[2] + (int32_t)z));
    const double2 *lut = static_cast<const double2 *>(a.lut64);
    r.rho = lut[clamp_hu<double>(a.hu[r.v])].x;
    if (a.mask && a.mask[r.v] == 0) r.rho = 0.0;
  }
  return r;
}

// tally / density: the dose up to factors common to the spot's voxels
__device__ __forceinline__ double inf_score(const InfEntry &x) {
  return (x.T > 0 && x.rho > 0.0) ? (double)x.T / x.rho : 0.0;
}

__device__ __forceinline__ bool inf_keep(const InfEntry &x, double thr) {
  return x.T > 0 && x.rho > 0.0 && (double)x.T / x.rho >= thr;
}

// Owner of tile t given the owner j of an earlier tile (tile_first is
// non-decreasing and tile_first[n_spots] = n_tiles > t).
__device__ __forceinline__ int advance_owner(const long long *tile_first, int j, long long t) {
  while (tile_first[j + 1] <= t) ++j;
  return j;
}

__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
  return x;
}

// Number of lanes of the wave for which `p` holds.
__device__ __forceinline__ uint32_t wave_count(bool p) { return (uint32_t)__popcll(__ballot(p)); }

// Per-thread maximum m of spot j -> the spot's maximum (atomic max on the bit
// pattern: non-negative doubles order like their bit patterns).
__device__ __forceinline__ void flush_spot_max(const InfluenceLaunch &a, int j, double m) {
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0 && m > 0.0)
    __hip_atomic_fetch_max(&a.spot_max[j], (unsigned long long)__double_as_longlong(m), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// The tally words of tile t for this thread: entries threadIdx.x + k kInfBlock
// of the tile.  Boxes lie back to back in whole tiles from the batch's first
// entry, so tile t starts at entry t kTile whatever spot owns it (padding
// entries are zero).
__device__ __forceinline__ void load_tile(const InfluenceLaunch &a, long long t, long long v[4]) {
  const long long *p = a.box_tally + t * kTile + threadIdx.x;
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = p[k * kInfBlock];
}

constexpr int kTilesAhead = 2;  // pass 1: tiles whose loads are in flight beyond the current one

// Pass 1 over a run of tiles per block: per spot, the maximum of
// tally / density; the 128-bit sum of all tallies; per tile, the number of
// nonzero entries (tile_count, zero before), so that later passes skip empty
// tiles and the last one clears exactly the tiles written.  Running values
// stay in registers: the block issues one max atomic per spot it meets and
// one sum atomic per wave, and no barrier.  The loads of the next
// kTilesAhead tiles are issued before the current tile is examined (most
// tiles are empty, and a tile's loads alone would leave the memory system
// idle between them).
__global__ void __launch_bounds__(kInfBlock) influence_max(InfluenceLaunch a, long long tiles_per_block) {
  const long long t_begin = (long long)blockIdx.x * tiles_per_block;
  const long long t_end = t_begin + tiles_per_block < a.n_tiles ? t_begin + tiles_per_block : a.n_tiles;
  if (t_begin >= t_end) return;
  int j = tile_owner(a.tile_first, a.n_spots, t_begin);
  BoxDev bx = a.boxes[j];
  long long tf = a.tile_first[j], tf_next = a.tile_first[j + 1];
  double m = 0.0;
  unsigned long long lo32 = 0, hi32 = 0;
  long long q[kTilesAhead + 1][4] = {};
#pragma unroll
  for (int i = 0; i <= kTilesAhead; ++i)
    if (t_begin + i < t_end) load_tile(a, t_begin + i, q[i]);
  for (long long t = t_begin; t < t_end; ++t) {
    long long cur[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) cur[k] = q[0][k];
#pragma unroll
    for (int i = 0; i < kTilesAhead; ++i)
#pragma unroll
      for (int k = 0; k < 4; ++k) q[i][k] = q[i + 1][k];
    if (t + kTilesAhead + 1 < t_end) load_tile(a, t + kTilesAhead + 1, q[kTilesAhead]);
    if (t >= tf_next) {  // block-uniform: the tile belongs to a later spot
      flush_spot_max(a, j, m);
      m = 0.0;
      j = advance_owner(a.tile_first, j, t);
      bx = a.boxes[j];
      tf = a.tile_first[j];
      tf_next = a.tile_first[j + 1];
    }
    const int32_t ne = bx.n[0] * bx.n[1] * bx.n[2];
    const int32_t e0 = (int32_t)((t - tf) * kTile);
    uint32_t nz = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int32_t e = e0 + (int32_t)threadIdx.x + k * kInfBlock;
      double sc = 0.0;
      if (e < ne) {
        const InfEntry x = inf_entry_of(a, bx, cur[k], e);
        sc = inf_score(x);
        const unsigned long long T = (unsigned long long)x.T;  // >= 0
        lo32 += T & 0xffffffffull;
        hi32 += T >> 32;
      }
      m = fmax(m, sc);
      nz += wave_count(cur[k] != 0);
    }
    if ((threadIdx.x & 63) == 0 && nz)
      __hip_atomic_fetch_add(&a.tile_count[t], nz, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  flush_spot_max(a, j, m);
  lo32 = wave_sum(lo32);  // < 2^32 entries of < 2^32 each per wave: no overflow
  hi32 = wave_sum(hi32);
  if ((threadIdx.x & 63) == 0) {
    const unsigned long long lo = lo32 + (hi32 << 32);
    const unsigned long long hi = (hi32 >> 32) + (lo < lo32 ? 1ull : 0ull);
    if (lo | hi) add128(a.dep_sum, lo, hi);
  }
}

// The tiles among [t0, t0 + 64) before t_end whose word in `per_tile` is
// nonzero, as a bit mask (bit i: tile t0 + i).  Every wave of the block reads
// the same words, so the mask is block-uniform.
__device__ __forceinline__ unsigned long long live_tiles(const uint32_t *per_tile, long long t0, long long t_end) {
  const long long t = t0 + (threadIdx.x & 63);
  const uint32_t c = t < t_end ? per_tile[t] : 0u;
  return __ballot(c != 0u);
}

// Pass 2: per tile, the number of entries at or above the spot's threshold
// (tile_keep, zero before).  The block reads the tile counts 64 at a time and
// visits only the tiles with energy.
__global__ void __launch_bounds__(kInfBlock) influence_count(InfluenceLaunch a, long long tiles_per_block) {
  const long long t_begin = (long long)blockIdx.x * tiles_per_block;
  const long long t_end = t_begin + tiles_per_block < a.n_tiles ? t_begin + tiles_per_block : a.n_tiles;
  if (t_begin >= t_end) return;
  int j = -1;
  for (long long t0 = t_begin; t0 < t_end; t0 += 64) {
    unsigned long long live = live_tiles(a.tile_count, t0, t_end);
    while (live) {
      const long long t = t0 + __builtin_ctzll(live);
      live &= live - 1;
      j = j < 0 ? tile_owner(a.tile_first, a.n_spots, t) : advance_owner(a.tile_first, j, t);
      const BoxDev bx = a.boxes[j];
      const int32_t ne = bx.n[0] * bx.n[1] * bx.n[2];
      const int32_t e0 = (int32_t)((t - a.tile_first[j]) * kTile);
      const double thr = a.rel_threshold * __longlong_as_double((long long)a.spot_max[j]);
      long long v[4];
      load_tile(a, t, v);
      uint32_t c = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int32_t e = e0 + (int32_t)threadIdx.x + k * kInfBlock;
        c += wave_count(e < ne && inf_keep(inf_entry_of(a, bx, v[k], e), thr));
      }
      if ((threadIdx.x & 63) == 0 && c)
        __hip_atomic_fetch_add(&a.tile_keep[t], c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// Inclusive scan of one value per thread over a block of 1024 threads;
// every thread must call it.  Returns the inclusive prefix and the total.
__device__ __forceinline__ unsigned long long block_scan_1024(unsigned long long x,
                                                              unsigned long long *total) {
  __shared__ unsigned long long wsum[16];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned long long y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  if (w == 0) {
    unsigned long long s = lane < 16 ? wsum[lane] : 0ull;
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
      const unsigned long long y = __shfl_up(s, o, 64);
      if (lane >= o) s += y;
    }
    if (lane < 16) wsum[lane] = s;
  }
  __syncthreads();
  const unsigned long long before = w > 0 ? wsum[w - 1] : 0ull;
  *total = wsum[15];
  __syncthreads();
  return x + before;
}

// exclusive offsets of the tiles within their chunk of 1024 tiles; chunk sums
__global__ void __launch_bounds__(1024) influence_scan_tiles(const uint32_t *tile_count, long long n_tiles,
                                                             unsigned long long *tile_off,
                                                             unsigned long long *chunk_sum) {
  const long long t = (long long)blockIdx.x * 1024 + threadIdx.x;
  const unsigned long long x = t < n_tiles ? tile_count[t] : 0ull;
  unsigned long long total;
  const unsigned long long incl = block_scan_1024(x, &total);
  if (t < n_tiles) tile_off[t] = incl - x;
  if (threadIdx.x == 0) chunk_sum[blockIdx.x] = total;
}

// chunk sums -> exclusive chunk offsets in place; chunk_off[n_chunks] = total
__global__ void __launch_bounds__(1024) influence_scan_chunks(unsigned long long *chunk_off,
                                                              long long n_chunks) {
  unsigned long long carry = 0;
  for (long long base = 0; base < n_chunks; base += 1024) {
    const long long c = base + threadIdx.x;
    const unsigned long long x = c < n_chunks ? chunk_off[c] : 0ull;
    unsigned long long total;
    const unsigned long long incl = block_scan_1024(x, &total);
    if (c < n_chunks) chunk_off[c] = carry + incl - x;
    carry += total;
  }
  if (threadIdx.x == 0) chunk_off[n_chunks] = carry;
}

__device__ __forceinline__ unsigned long long tile_offset(const InfluenceLaunch &a, long long t) {
  const long long n_chunks = (a.n_tiles + 1023) / 1024;
  return t < a.n_tiles ? a.chunk_off[t >> 10] + a.tile_off[t] : a.chunk_off[n_chunks];
}

// Pass 4: entries of the tile at or above the threshold, in entry order, at
// the tile's offset.  A block owns kWriteTiles consecutive tiles, reads
// their kept counts at once and visits only the tiles with kept entries.
__global__ void __launch_bounds__(kInfBlock) influence_write(InfluenceLaunch a) {
  __shared__ uint32_t wcount[kInfBlock / 64];
  const long long t_begin = (long long)blockIdx.x * kWriteTiles;
  const long long t_end = t_begin + kWriteTiles < a.n_tiles ? t_begin + kWriteTiles : a.n_tiles;
  unsigned long long live = live_tiles(a.tile_keep, t_begin, t_end);  // block-uniform
  int j = -1;
  while (live) {
    const long long t = t_begin + __builtin_ctzll(live);
    live &= live - 1;
    j = j < 0 ? tile_owner(a.tile_first, a.n_spots, t) : advance_owner(a.tile_first, j, t);
    const BoxDev bx = a.boxes[j];
    const int32_t ne = bx.n[0] * bx.n[1] * bx.n[2];
    const int32_t e0 = (int32_t)((t - a.tile_first[j]) * kTile);
    const double thr = a.rel_threshold * __longlong_as_double((long long)a.spot_max[j]);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    unsigned long long pos = (unsigned long long)a.nnz_base + tile_offset(a, t);
    long long v[4];
    load_tile(a, t, v);
    for (int k = 0; k < 4; ++k) {  // sub-tiles of 256 consecutive entries, in order
      const int32_t e = e0 + (int32_t)threadIdx.x + k * kInfBlock;
      InfEntry x = {};
      bool keep = false;
      if (e < ne) {
        x = inf_entry_of(a, bx, v[k], e);
        keep = inf_keep(x, thr);
      }
      const unsigned long long bal = __ballot(keep);
      const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
      if (lane == 0) wcount[w] = (uint32_t)__popcll(bal);
      __syncthreads();
      uint32_t before = 0, sub = 0;
      for (int i = 0; i < kInfBlock / 64; ++i) {
        before += i < w ? wcount[i] : 0u;
        sub += wcount[i];
      }
      if (keep) {
        const unsigned long long p = pos + before + rank;
        const double e_j = (double)x.T / 4294967296.0 * 1.602176634e-13;
        const double m_kg = x.rho * a.vol_cm3 * 1e-3;
        a.voxel[p] = x.v;
        a.value[p] = (float)(e_j / m_kg / bx.n_hist);
      }
      pos += sub;
      __syncthreads();
    }
  }
}

// After pass 4: every tile with a nonzero entry back to zero, so that the
// box tallies need no full fill before the next batch.
__global__ void __launch_bounds__(kInfBlock) influence_clear(InfluenceLaunch a) {
  const long long t_begin = (long long)blockIdx.x * kWriteTiles;
  const long long t_end = t_begin + kWriteTiles < a.n_tiles ? t_begin + kWriteTiles : a.n_tiles;
  unsigned long long live = live_tiles(a.tile_count, t_begin, t_end);
  long long *tally = const_cast<long long *>(a.box_tally);
  while (live) {
    const long long t = t_begin + __builtin_ctzll(live);
    live &= live - 1;
    long long *p = tally + t * kTile + threadIdx.x;
#pragma unroll
    for (int k = 0; k < 4; ++k) p[k * kInfBlock] = 0;
  }
}

__global__ void influence_rows(InfluenceLaunch a) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < a.n_spots) a.row_ptr[j] = a.nnz_base + (long long)tile_offset(a, a.tile_first[j]);
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

template <typename R, bool LUT_LDS, bool BOX>
static void launch_persistent_v(const PersistentLaunch &a, size_t lds, hipStream_t st) {
  using R2 = typename M<R>::R2;
  using R4 = typename M<R>::R4;
  hipLaunchKernelGGL((transport_persistent<R, LUT_LDS, BOX>), dim3(a.grid), dim3(a.block), lds, st,
                     (const SpotDev<R> *)a.spots, a.items, a.n_items, a.targets, a.n_targets,
                     (const R2 *)a.luts, (const R4 *)a.tab, (R)a.l2e0, (R)a.inv_dl2, (R)a.dl2,
                     a.k0, a.k1, a.flags, a.refill_min, a.cursor, a.counters, a.boxes,
                     a.box_tally, a.box_bias, a.drained);
}

template <typename R>
static hipError_t launch_core_t(const PersistentLaunch &a, hipStream_t st) {
  if constexpr (sizeof(R) != sizeof(float)) {
    return hipErrorInvalidValue;  // the block engine runs in FP32 only
  } else {
    using R2 = typename M<R>::R2;
    using R4 = typename M<R>::R4;
    const size_t lds = core_fixed_lds(a.lut_lds) + sizeof(unsigned long long) * (size_t)a.core_cap;
    const bool box = a.boxes != nullptr;
    if (a.log && (box || !a.lut_lds)) return hipErrorInvalidValue;  // logged: phase tallies, one LUT
    // slice cores that follow an oblique beam need the general key; cores
    // that are all boxes of the grid take the cheaper one
    const bool sl = a.slanted;
    auto kern = a.log ? (sl ? transport_core<R, true, false, true, true> : transport_core<R, true, false, true>)
              : a.lut_lds ? (box ? (sl ? transport_core<R, true, true, false, true> : transport_core<R, true, true>)
                                 : (sl ? transport_core<R, true, false, false, true> : transport_core<R, true, false>))
                          : (box ? (sl ? transport_core<R, false, true, false, true> : transport_core<R, false, true>)
                                 : (sl ? transport_core<R, false, false, false, true> : transport_core<R, false, false>));
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(a.grid), dim3(kCoreBlock), lds, st, (const SpotDev<R> *)a.spots,
                       a.items, a.n_items, a.targets, (const R2 *)a.luts, (const R4 *)a.tab,
                       (R)a.l2e0, (R)a.inv_dl2, (R)a.dl2, a.k0, a.k1, a.flags, a.refill_min, a.cursor,
                       a.counters, a.slices, a.cores, a.core_cap, a.boxes, a.box_tally, a.box_bias, a.drained,
                       a.log, a.log_cap, a.log_count);
    return hipGetLastError();
  }
}

template <typename R>
static hipError_t launch_persistent_t(const PersistentLaunch &a, hipStream_t st) {
  if (a.cores || a.slices) return launch_core_t<R>(a, st);
  const size_t lds = persistent_lds<R>(a);
  const bool box = a.boxes != nullptr;
  if (a.lut_lds && box) launch_persistent_v<R, true, true>(a, lds, st);
  else if (a.lut_lds) launch_persistent_v<R, true, false>(a, lds, st);
  else if (box) launch_persistent_v<R, false, true>(a, lds, st);
  else launch_persistent_v<R, false, false>(a, lds, st);
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
  const size_t lds = persistent_lds<R>(a);
  const bool box = a.boxes != nullptr;
  if (a.lut_lds && box)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, transport_persistent<R, true, true>, a.block, lds);
  else if (a.lut_lds)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, transport_persistent<R, true, false>, a.block, lds);
  else if (box)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, transport_persistent<R, false, true>, a.block, lds);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, transport_persistent<R, false, false>, a.block, lds);
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

hipError_t launch_influence_reduce(const InfluenceLaunch &a, hipStream_t st) {
  const long long n_chunks = (a.n_tiles + 1023) / 1024;
  if (a.n_tiles > 0) {
    // the reduction passes in a few thousand blocks of consecutive tiles
    const long long per = (a.n_tiles + 4095) / 4096;
    const unsigned blocks = (unsigned)((a.n_tiles + per - 1) / per);
    hipLaunchKernelGGL(influence_max, dim3(blocks), dim3(kInfBlock), 0, st, a, per);
    hipLaunchKernelGGL(influence_count, dim3(blocks), dim3(kInfBlock), 0, st, a, per);
    hipLaunchKernelGGL(influence_scan_tiles, dim3((unsigned)n_chunks), dim3(1024), 0, st,
                       (const uint32_t *)a.tile_keep, a.n_tiles, a.tile_off, a.chunk_off);
  }
  hipLaunchKernelGGL(influence_scan_chunks, dim3(1), dim3(1024), 0, st, a.chunk_off, n_chunks);
  return hipGetLastError();
}

hipError_t launch_influence_write(const InfluenceLaunch &a, hipStream_t st) {
  const unsigned blocks = (unsigned)((a.n_tiles + kWriteTiles - 1) / kWriteTiles);
  if (a.n_tiles > 0) {
    hipLaunchKernelGGL(influence_write, dim3(blocks), dim3(kInfBlock), 0, st, a);
    hipLaunchKernelGGL(influence_clear, dim3(blocks), dim3(kInfBlock), 0, st, a);
  }
  if (a.n_spots > 0)
    hipLaunchKernelGGL(influence_rows, dim3((unsigned)((a.n_spots + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_atomic_replay(const unsigned long long *log, uint32_t log_cap, const uint32_t *log_count,
                                uint32_t n_lanes, hipStream_t st) {
  if (n_lanes == 0) return hipSuccess;
  hipLaunchKernelGGL(atomic_replay, dim3((n_lanes + kCoreBlock - 1) / kCoreBlock), dim3(kCoreBlock), 0, st,
                     log, log_cap, log_count, n_lanes);
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

// ---------------------------------------------------------------------------
// scratch of the no-allocation entry point: one array per device, whose
// address host code takes once per device with hipGetSymbolAddress (the
// array's name is not a device address in host code)
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mutex;
NoAlloc g_noalloc[kMaxDevices];
}  // namespace

hipError_t noalloc_setup(int device, NoAlloc **out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_noalloc_mutex);
  NoAlloc &na = g_noalloc[device];
  if (!na.dev) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    void *h = nullptr;
    e = hipHostMalloc(&h, kNoAllocBytes, hipHostMallocDefault);
    if (e != hipSuccess) return e;
    hipEvent_t ev = nullptr;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) {
      (void)hipHostFree(h);
      return e;
    }
    na.dev = static_cast<unsigned char *>(p);
    na.host = static_cast<unsigned char *>(h);
    na.uploaded = ev;
  }
  *out = &na;
  return hipSuccess;
}

}  // namespace pmc
