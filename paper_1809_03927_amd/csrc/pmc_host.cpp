// C ABI of libpmc (include/pmc.h): argument validation, ownership of device
// memory, the history split and work decomposition, kernel launches and the
// energy balance.
//
// Inputs follow the paper's statement of the problem: a CT per breathing
// phase with its HU -> density conversion (Sec. 2.C), an optional external
// contour bounding transport (Sec. 2.A), and plan spots (position, energy,
// weight; Appendix A) distributed over phases by the delivery simulation
// (Sec. 2.B).  Outputs are dose and density per CT voxel (Sec. 2.C).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "pmc.h"
#include "pmc_internal.hpp"

using pmc::SpotDev;
using pmc::TargetDev;
using pmc::WorkItem;

namespace {

thread_local std::string g_error;  // message for failures without a context

constexpr int kHuLo = -1024, kHuHi = 3071, kLut = 4096;
constexpr int kMaxPhaseId = 1023;
constexpr double kTwo32 = 4294967296.0;

constexpr int kCursorSlots = 16;

struct DevBuf {
  void *p = nullptr;
  size_t cap = 0;
};

// Events recorded, per stream, after the latest enqueued work that reads a
// resource; freeing or rewriting the resource waits for them only.
struct UseEvents {
  std::vector<std::pair<hipStream_t, hipEvent_t>> ev;
};

struct PhaseRec {
  int32_t nx = 0, ny = 0, nz = 0;
  double sp_mm[3] = {0, 0, 0}, org_mm[3] = {0, 0, 0};
  std::vector<float> lut32;   // (rho, rsp) x 4096
  std::vector<double> lut64;  // (rho, rsp) x 4096
  bool has_mask = false;
  uint64_t version = 0;
  int16_t *d_hu = nullptr;
  uint8_t *d_mask = nullptr;
  void *d_lut32 = nullptr, *d_lut64 = nullptr;
  size_t cap_hu = 0, cap_mask = 0, cap_lut32 = 0, cap_lut64 = 0;  // pool block sizes
  size_t bytes = 0;
  UseEvents uses;
  std::vector<int16_t> hu_host;     // host copies for geometry queries (influence boxes)
  std::vector<uint8_t> mask_host;
  long long nvox() const { return (long long)nx * ny * nz; }
};

// A resident deformation vector field (App. B).
struct DvfRec {
  pmc::DvfDev dev = {};   // geometry; dev.delta points into d_delta
  void *d_delta = nullptr;
  size_t cap = 0;
  size_t bytes = 0;
  UseEvents uses;
};

struct PlanRec {
  std::vector<pmc_field> fields;
  std::vector<pmc_spot> spots;
  uint64_t version = 0;
};

// Device-side data of a request that depends only on its inputs (plan,
// phases, split, engine); kept in a small LRU cache of such entries.
struct Prepared {
  // signature
  int32_t plan_id = -1;
  uint64_t plan_version = 0, n_hist = 0;
  std::vector<int32_t> phases;
  std::vector<uint64_t> phase_versions;
  int32_t engine = -1, chunk = -1, precision = -1, mode = 0;
  // host side
  std::vector<int64_t> per_spot;
  std::vector<std::vector<int32_t>> list;      // per slot: spots with histories
  std::vector<std::vector<long long>> first;   // per slot: prefix offsets
  std::vector<long long> slot_hist;
  int32_t n_items = 0;
  bool same_lut = true;
  unsigned __int128 incident = 0;
  // device offsets into the request scratch buffer
  size_t off_spots = 0, off_items = 0, off_luts = 0, off_targets = 0, off_cores = 0;
  int32_t core_cap = 0;  // PMC_TALLY_CORE: LDS tally entries per block
  bool slanted = false;  // PMC_TALLY_CORE: some slice core follows an oblique beam
  std::vector<size_t> off_ids, off_first;
  std::vector<unsigned char> staging;  // host image uploaded into the scratch
  std::vector<TargetDev> targets;      // last uploaded target table
  size_t bytes = 0;                    // size of the request data
  DevBuf buf;                          // device copy of the request data
  uint64_t last_use = 0;
  UseEvents uses;
};

}  // namespace

struct pmc_graph {
  pmc_context *ctx = nullptr;
  std::vector<int32_t> phases;  // phases the graph's kernels read
  std::vector<uint64_t> versions;  // their versions at capture: the graph holds their device pointers
  void *data = nullptr;  // private copy of the request data + work-queue cursor
  size_t bytes = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

struct pmc_context {
  int device = -1;
  int precision = PMC_FP32;
  uint64_t seed = 0;
  uint64_t budget = 0;
  uint64_t used = 0;
  bool has_device = false;
  int n_cu = 0;
  size_t lds_max = 160 * 1024;  // LDS bytes a block may use (device property)
  std::string err;
  pmc::Tables tabs;
  void *d_tab = nullptr;
  size_t tab_bytes = 0;
  std::map<int32_t, PhaseRec> phases;
  uint64_t phase_counter = 0;
  std::map<int32_t, PlanRec> plans;
  uint64_t plan_counter = 0;
  hipStream_t stream = nullptr;
  // Freed device blocks kept for reuse, by (rounded) size: hipFree waits for
  // the whole device, which would stall work running on other streams.
  // Pooled blocks count as used; they are freed when the budget needs room.
  std::multimap<size_t, void *> pool;
  // Work enqueued on callers' streams: one event per stream, recorded after
  // the stream's latest enqueue; all are waited for before device memory
  // that such work may read is freed or overwritten.
  std::map<hipStream_t, hipEvent_t> stream_done;
  std::vector<std::unique_ptr<Prepared>> cache;  // prepared request data (LRU)
  uint64_t use_counter = 0;
  // Work-queue cursors of persistent launches, one 256-byte line each, used
  // round robin; a launch that reuses a cursor first waits (on the device)
  // for the launch that used it before, so launches on different streams may
  // run concurrently.
  DevBuf cursor;
  hipEvent_t cursor_done[kCursorSlots] = {};
  int next_cursor = 0;
  DevBuf counters;   // internal counter block
  // influence calculations: box tallies of a batch of spots, bookkeeping,
  // and the result (CSR rows, one per plan spot)
  DevBuf box_scratch, inf_work;
  // leading entries of box_scratch known to be zero: every influence batch
  // clears the tiles it wrote, so later batches need not zero them again
  long long box_zero = 0;
  DevBuf inf_rows, inf_voxel, inf_value;
  size_t inf_cap = 0;        // capacity of inf_voxel / inf_value, entries
  int64_t inf_n_rows = -1;   // -1: no result
  uint64_t inf_nnz = 0;
  // dose accumulation: resident DVFs and the energy/mass accumulators of the
  // reference grid (3 x uint64 per voxel), last used on the streams in acc_uses
  std::map<int32_t, DvfRec> dvfs;
  DevBuf acc;
  UseEvents acc_uses;
  // pmc_dose_device_noalloc: the device's scratch array (shared by every
  // context on the device) and whether a call since the last device-wide
  // wait may still read the context's phases or tables
  pmc::NoAlloc *noalloc = nullptr;
  bool noalloc_used = false;
};

namespace {

int fail(pmc_context *ctx, int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (ctx) ctx->err = buf;
  else g_error = buf;
  return code;
}

int hip_fail(pmc_context *ctx, hipError_t e, const char *what) {
  return fail(ctx, PMC_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(ctx, call, what)                      \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, what); \
  } while (0)

bool finite3(const double v[3]) {
  return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]);
}

double norm3(const double v[3]) { return std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); }

// piecewise-linear calibration at an integer HU, clamped to the end nodes
double calib_at(const double *x, const double *y, int n, double hu) {
  if (hu <= x[0]) return y[0];
  if (hu >= x[n - 1]) return y[n - 1];
  int i = (int)(std::upper_bound(x, x + n, hu) - x) - 1;  // x[i] <= hu < x[i+1]
  const double t = (hu - x[i]) / (x[i + 1] - x[i]);
  return y[i] + (y[i + 1] - y[i]) * t;
}

void wait_pending(pmc_context *ctx);

// Sizes handed out by the pool: powers of two up to 1 MiB, then multiples
// of 2 MiB, so that freed blocks fit later requests of similar size.
size_t pool_round(size_t n) {
  if (n <= (size_t(1) << 20)) {
    size_t p = 256;
    while (p < n) p <<= 1;
    return p;
  }
  const size_t g = size_t(2) << 20;
  return (n + g - 1) / g * g;
}

// Free every pooled block (hipFree: waits for the device).
void trim_pool(pmc_context *ctx) {
  for (auto &kv : ctx->pool) {
    (void)hipFree(kv.second);
    ctx->used -= kv.first;
  }
  ctx->pool.clear();
}

// A device block of at least n bytes (*cap = its size): a pooled block of
// the same rounded size, or a new one within the budget.
int pool_get(pmc_context *ctx, size_t n, void **out, size_t *cap, const char *what) {
  const size_t r = pool_round(std::max<size_t>(n, 1));
  auto it = ctx->pool.find(r);
  if (it != ctx->pool.end()) {
    *out = it->second;
    *cap = r;
    ctx->pool.erase(it);
    return PMC_OK;
  }
  if (ctx->used + r > ctx->budget) trim_pool(ctx);
  if (ctx->used + r > ctx->budget)
    return fail(ctx, PMC_E_BUDGET, "%s: %zu bytes exceed the device-memory budget (%llu in use of %llu)",
                what, r, (unsigned long long)ctx->used, (unsigned long long)ctx->budget);
  void *p = nullptr;
  HIP_TRY(ctx, hipMalloc(&p, r), what);
  ctx->used += r;
  *out = p;
  *cap = r;
  return PMC_OK;
}

// Return a block to the pool.  No enqueued work may still use it.
void pool_put(pmc_context *ctx, void *p, size_t cap) {
  if (p) ctx->pool.emplace(cap, p);
}

// grow-only device buffer with budget accounting
int ensure(pmc_context *ctx, DevBuf &b, size_t bytes, const char *what) {
  if (b.cap >= bytes) return PMC_OK;
  if (b.p) {
    wait_pending(ctx);  // context buffers may be read by enqueued work
    pool_put(ctx, b.p, b.cap);
    b.p = nullptr;
    b.cap = 0;
  }
  return pool_get(ctx, std::max(bytes, b.cap + b.cap / 2), &b.p, &b.cap, what);
}

// Give a buffer back to the pool; the caller has waited for its users.
void release(pmc_context *ctx, DevBuf &b) {
  pool_put(ctx, b.p, b.cap);
  b.p = nullptr;
  b.cap = 0;
}

// Copy through the context's own stream (non-blocking with respect to every
// other stream, unlike a synchronous copy on the null stream) and wait.
hipError_t copy_sync(pmc_context *ctx, void *dst, const void *src, size_t bytes, hipMemcpyKind kind) {
  hipError_t e = hipMemcpyAsync(dst, src, bytes, kind, ctx->stream);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(ctx->stream);
}

int note_use(pmc_context *ctx, UseEvents &u, hipStream_t st) {
  for (auto &p : u.ev)
    if (p.first == st) {
      HIP_TRY(ctx, hipEventRecord(p.second, st), "hipEventRecord");
      return PMC_OK;
    }
  hipEvent_t e = nullptr;
  HIP_TRY(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
  u.ev.emplace_back(st, e);
  HIP_TRY(ctx, hipEventRecord(e, st), "hipEventRecord");
  return PMC_OK;
}

void wait_use(UseEvents &u) {
  for (auto &p : u.ev) (void)hipEventSynchronize(p.second);
}

void drop_use(UseEvents &u) {
  for (auto &p : u.ev) (void)hipEventDestroy(p.second);
  u.ev.clear();
}

// Work of pmc_dose_device_noalloc records no per-resource events (creating
// one is itself a setup call); memory it may read is released only after a
// device-wide wait.
void wait_noalloc(pmc_context *ctx) {
  if (!ctx->noalloc_used) return;
  (void)hipDeviceSynchronize();
  ctx->noalloc_used = false;
}

void free_phase(pmc_context *ctx, PhaseRec &p) {
  wait_noalloc(ctx);
  wait_use(p.uses);
  drop_use(p.uses);
  pool_put(ctx, p.d_hu, p.cap_hu);
  pool_put(ctx, p.d_mask, p.cap_mask);
  pool_put(ctx, p.d_lut32, p.cap_lut32);
  pool_put(ctx, p.d_lut64, p.cap_lut64);
  p.d_hu = nullptr;
  p.d_mask = nullptr;
  p.d_lut32 = p.d_lut64 = nullptr;
  p.bytes = 0;
}

void wait_pending(pmc_context *ctx) {
  for (auto &kv : ctx->stream_done) (void)hipEventSynchronize(kv.second);
}

// Record that work reading the context's device memory was enqueued on st.
int note_pending(pmc_context *ctx, hipStream_t st) {
  hipEvent_t &ev = ctx->stream_done[st];
  if (!ev) HIP_TRY(ctx, hipEventCreateWithFlags(&ev, hipEventDisableTiming), "hipEventCreate");
  HIP_TRY(ctx, hipEventRecord(ev, st), "hipEventRecord");
  return PMC_OK;
}

long long q_working(const pmc_context *ctx, double E) {
  if (ctx->precision == PMC_FP32) return (long long)std::ldexp((double)(float)E, 32);
  return std::llrint(E * kTwo32);
}

int split(const pmc_spot *spots, int64_t n_spots, const int32_t *phases, int32_t n_phases,
          uint64_t n_hist, int64_t *per_spot) {
  auto listed = [&](int32_t ph) {
    for (int32_t i = 0; i < n_phases; ++i)
      if (phases[i] == ph) return true;
    return false;
  };
  double W = 0.0;
  std::vector<int64_t> members;
  for (int64_t s = 0; s < n_spots; ++s) {
    per_spot[s] = 0;
    if (listed(spots[s].phase)) {
      W += spots[s].weight;
      members.push_back(s);
    }
  }
  if (members.empty() || !(W > 0.0)) return PMC_E_INVAL;
  std::vector<std::pair<double, int64_t>> rem;
  rem.reserve(members.size());
  uint64_t given = 0;
  for (int64_t s : members) {
    const double share = (double)n_hist * spots[s].weight / W;
    const double whole = std::floor(share);
    per_spot[s] = (int64_t)whole;
    given += (uint64_t)whole;
    rem.emplace_back(share - whole, s);
  }
  std::stable_sort(rem.begin(), rem.end(), [](const std::pair<double, int64_t> &a,
                                              const std::pair<double, int64_t> &b) {
    return a.first > b.first || (a.first == b.first && a.second < b.second);
  });
  uint64_t left = n_hist > given ? n_hist - given : 0;
  for (size_t k = 0; k < rem.size() && left > 0; ++k, --left) per_spot[rem[k].second] += 1;
  return PMC_OK;
}

int validate_request(pmc_context *ctx, const pmc_request *req) {
  if (!req) return fail(ctx, PMC_E_INVAL, "request is NULL");
  auto pit = ctx->plans.find(req->plan);
  if (pit == ctx->plans.end())
    return fail(ctx, PMC_E_STATE, "plan %d is not loaded (call pmc_load_plan / pmc_load_spots first)",
                req->plan);
  if (req->n_phases < 1 || req->n_phases > PMC_MAX_PHASES || !req->phases)
    return fail(ctx, PMC_E_INVAL, "n_phases must be 1..%d with a phase list", PMC_MAX_PHASES);
  for (int32_t i = 0; i < req->n_phases; ++i) {
    if (!ctx->phases.count(req->phases[i]))
      return fail(ctx, PMC_E_NOPHASE, "phase %d is not loaded", req->phases[i]);
    for (int32_t j = 0; j < i; ++j)
      if (req->phases[j] == req->phases[i])
        return fail(ctx, PMC_E_INVAL, "phase %d listed twice", req->phases[i]);
  }
  if (req->n_histories == 0) return fail(ctx, PMC_E_INVAL, "n_histories must be >= 1");
  if (req->n_histories > PMC_MAX_HISTORIES)
    return fail(ctx, PMC_E_RANGE, "n_histories %llu exceeds %llu per tally",
                (unsigned long long)req->n_histories, (unsigned long long)PMC_MAX_HISTORIES);
  if (req->engine != PMC_ENGINE_PLAIN && req->engine != PMC_ENGINE_PERSISTENT)
    return fail(ctx, PMC_E_INVAL, "unknown engine %d", req->engine);
  if (req->block_size != 0 && (req->block_size < 64 || req->block_size > 1024 || req->block_size % 64))
    return fail(ctx, PMC_E_INVAL, "block_size must be 0 or a multiple of 64 in [64, 1024]");
  if (ctx->precision == PMC_FP64 && req->block_size > 256)
    return fail(ctx, PMC_E_INVAL, "FP64 kernels take at most 256 threads per block");
  if (req->chunk < 0 || req->refill_min < 0 || req->refill_min > 64 || req->grid_blocks < 0)
    return fail(ctx, PMC_E_INVAL, "chunk, refill_min (0..64) and grid_blocks must be >= 0");
  if (req->flags & ~31u) return fail(ctx, PMC_E_INVAL, "unknown flag bits 0x%x", req->flags);
  if (req->tally_mode < PMC_TALLY_AUTO || req->tally_mode > PMC_TALLY_CORE)
    return fail(ctx, PMC_E_INVAL, "unknown tally_mode %d", req->tally_mode);
  if (req->tally_mode == PMC_TALLY_CORE) {
    if (req->engine != PMC_ENGINE_PERSISTENT || ctx->precision != PMC_FP32)
      return fail(ctx, PMC_E_INVAL, "PMC_TALLY_CORE needs the FP32 persistent engine");
    if (req->block_size != 0 && req->block_size != pmc::kCoreBlock)
      return fail(ctx, PMC_E_INVAL, "PMC_TALLY_CORE runs %d threads per block", pmc::kCoreBlock);
  }
  if (req->engine == PMC_ENGINE_PLAIN && (req->item_begin || req->item_end))
    return fail(ctx, PMC_E_INVAL, "work-item slices need the persistent engine");
  if (req->item_end && req->item_end < req->item_begin)
    return fail(ctx, PMC_E_INVAL, "item_end < item_begin");
  bool any = false;
  for (const pmc_spot &s : pit->second.spots)
    for (int32_t i = 0; i < req->n_phases && !any; ++i) any = s.phase == req->phases[i];
  if (!any) return fail(ctx, PMC_E_INVAL, "no spot of the plan lies on the requested phases");
  return PMC_OK;
}

template <typename R>
SpotDev<R> make_spot(const pmc_spot &s, const pmc_field &f, const PhaseRec &ph, int32_t target) {
  double w[3], u[3], v[3];
  const double nw = norm3(f.direction), nu = norm3(f.bev_u);
  for (int k = 0; k < 3; ++k) {
    w[k] = f.direction[k] / nw;
    u[k] = f.bev_u[k] / nu;
  }
  v[0] = w[1] * u[2] - w[2] * u[1];
  v[1] = w[2] * u[0] - w[0] * u[2];
  v[2] = w[0] * u[1] - w[1] * u[0];
  SpotDev<R> d;
  for (int k = 0; k < 3; ++k) {
    const double c = 0.1 * (f.isocentre_mm[k] - ph.org_mm[k]) + 0.1 * s.x_mm * u[k] + 0.1 * s.y_mm * v[k];
    d.c[k] = (R)c;
    d.u[k] = (R)u[k];
    d.v[k] = (R)v[k];
    d.w[k] = (R)w[k];
  }
  d.sigma = (R)(0.1 * s.sigma_mm);
  d.E = (R)s.energy_MeV;
  d.target = target;
  d.pad = 0;
  return d;
}

TargetDev make_target(const PhaseRec &ph, unsigned long long *tally, int32_t lut) {
  TargetDev t;
  t.hu = ph.d_hu;
  t.mask = ph.d_mask;
  t.tally = tally;
  t.nx = ph.nx;
  t.ny = ph.ny;
  t.nz = ph.nz;
  t.lut = lut;
  for (int k = 0; k < 3; ++k) t.d[k] = 0.1 * ph.sp_mm[k];
  return t;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// f(i) for i in [0, n) on up to 16 host threads (f must be safe to run
// concurrently for different i); small n runs inline.
template <typename F>
void parallel_for(int64_t n, F &&f) {
  const unsigned hw = std::thread::hardware_concurrency();
  const int64_t nt = std::min<int64_t>(hw ? hw : 1, 16);
  if (n < 512 || nt <= 1) {
    for (int64_t i = 0; i < n; ++i) f(i);
    return;
  }
  std::atomic<int64_t> next{0};
  auto work = [&]() {
    for (;;) {
      const int64_t i0 = next.fetch_add(64);
      if (i0 >= n) return;
      const int64_t i1 = std::min<int64_t>(n, i0 + 64);
      for (int64_t i = i0; i < i1; ++i) f(i);
    }
  };
  std::vector<std::thread> pool;
  for (int64_t t = 1; t < nt; ++t) pool.emplace_back(work);
  work();
  for (auto &t : pool) t.join();
}

// Launch shape of a request: its own values where set, else the defaults.
// Threads per block: 1024 for the FP32 persistent engine (one block fills a
// CU's wave slots that the LDS tables and registers allow: 16 waves), the
// launch bound 256 for FP64 and for the plain engine.  Histories per work
// item (lane mode): the largest of 256, 128, 64 that still hands each
// resident wave about four items, so that a small request spreads over the
// whole device instead of running several histories in a row on the lanes of
// a few waves.  Core mode: items of 8192 histories (8 per lane of a block),
// so that the wait of a block's waves for its item's last history, and the
// flush of the core, are small against the item.
struct LaunchShape {
  int32_t block, chunk, refill, mode, core_cap;
};

constexpr int32_t kCoreChunk = 8192;
constexpr int32_t kCoreMinEntries = 4096;

bool same_lut(const pmc_context *ctx, const pmc_request *req) {
  for (int32_t i = 1; i < req->n_phases; ++i)
    if (ctx->phases.at(req->phases[i]).lut64 != ctx->phases.at(req->phases[0]).lut64) return false;
  return true;
}

int32_t core_capacity(const pmc_context *ctx, bool lut_lds) {
  const size_t fixed = pmc::core_fixed_lds(lut_lds);
  if (ctx->lds_max <= fixed) return 0;
  return (int32_t)std::min<size_t>((ctx->lds_max - fixed) / sizeof(unsigned long long), 1u << 30);
}

// Requires a validated request.
// Histories per work item of the block engine: kCoreChunk (8 per lane of a
// block), halved down to one per lane while the request has fewer than that
// per CU (small requests: more, shorter items spread over more CUs).
int32_t core_chunk(const pmc_context *ctx, const pmc_request *req) {
  if (req->chunk > 0) return req->chunk;
  const int64_t n_cu = ctx->n_cu > 0 ? ctx->n_cu : 256;
  const int64_t per_cu = (int64_t)(req->n_histories / (uint64_t)n_cu);
  int32_t c = kCoreChunk;
  while (c > pmc::kCoreBlock && c > per_cu) c >>= 1;
  return c;
}

LaunchShape launch_shape(const pmc_context *ctx, const pmc_request *req) {
  const bool persistent = req->engine == PMC_ENGINE_PERSISTENT;
  const bool fp32 = ctx->precision != PMC_FP64;
  LaunchShape s;
  s.refill = persistent ? (req->refill_min ? req->refill_min : 64) : 0;
  s.mode = persistent ? req->tally_mode : 0;
  s.core_cap = 0;
  const int64_t n_cu = ctx->n_cu > 0 ? ctx->n_cu : 256;
  if (persistent && s.mode == PMC_TALLY_AUTO) {
    s.mode = PMC_TALLY_LANE;
    const int32_t cap = fp32 ? core_capacity(ctx, same_lut(ctx, req)) : 0;
    if (cap >= kCoreMinEntries && (req->block_size == 0 || req->block_size == pmc::kCoreBlock)) {
      // the mode is decided on items of kCoreChunk (or the given chunk); a
      // small request then gets shorter items (core_chunk)
      const int64_t chunk = req->chunk > 0 ? req->chunk : kCoreChunk;
      const std::vector<pmc_spot> &sp = ctx->plans.at(req->plan).spots;
      std::vector<int64_t> per(sp.size(), 0);
      if (split(sp.data(), (int64_t)sp.size(), req->phases, req->n_phases, req->n_histories, per.data()) == 0) {
        // at least one history per lane of a block per item on average
        // (counting a spot's partial last item with its full ones): spots
        // with fewer histories spread better over the lanes of many waves
        // (lane engine)
        int64_t items = 0;
        for (int64_t h : per)
          if (h > 0) items += std::max<int64_t>(1, h / chunk);
        if ((int64_t)req->n_histories >= (int64_t)pmc::kCoreBlock * items) s.mode = PMC_TALLY_CORE;
      }
    }
  }
  if (s.mode == PMC_TALLY_CORE) {
    s.block = pmc::kCoreBlock;
    s.chunk = core_chunk(ctx, req);
    s.core_cap = core_capacity(ctx, same_lut(ctx, req));
    return s;
  }
  s.block = req->block_size ? req->block_size : (persistent && fp32 ? 1024 : 256);
  s.chunk = 0;
  if (persistent) {
    if (req->chunk > 0) {
      s.chunk = req->chunk;
    } else {
      const uint64_t waves = 16ull * (uint64_t)n_cu;
      s.chunk = 256;
      while (s.chunk > 64 && req->n_histories < 4ull * waves * (uint64_t)s.chunk) s.chunk >>= 1;
    }
  }
  return s;
}

int default_chunk(const pmc_context *ctx, const pmc_request *req) { return launch_shape(ctx, req).chunk; }

pmc_box spot_box(const pmc_context *ctx, const PhaseRec &ph, const pmc_field &f, const pmc_spot &s);
pmc::SliceCore slice_core(const pmc_context *ctx, const PhaseRec &ph, const pmc_field &f, const pmc_spot &s,
                          int32_t cap, const pmc_box *inside = nullptr);

// Core box of a spot: its voxel box if that fits `cap` entries, else the box's
// full extent along the beam's main axis and a window across it, centred in
// the box, with the box's aspect ratio and at most `cap` entries in all.
pmc::CoreDev core_of(const pmc_box &b, const pmc_field &f, int32_t cap) {
  pmc::CoreDev c = {};
  int64_t n[3];
  for (int k = 0; k < 3; ++k) {
    c.lo[k] = b.lo[k];
    n[k] = b.hi[k] > b.lo[k] ? b.hi[k] - b.lo[k] : 0;
  }
  if (n[0] * n[1] * n[2] == 0 || cap <= 0) return c;
  if (n[0] * n[1] * n[2] > cap) {
    int d = 0;
    for (int k = 1; k < 3; ++k)
      if (std::fabs(f.direction[k]) > std::fabs(f.direction[d])) d = k;
    const int a = (d + 1) % 3, e = (d + 2) % 3;
    const int64_t cells = cap / n[d];
    if (cells < 1) return c;  // not even the axis fits: no core
    int64_t wa = (int64_t)std::floor(std::sqrt((double)cells * (double)n[a] / (double)n[e]));
    wa = std::max<int64_t>(1, std::min(wa, n[a]));
    int64_t we = std::max<int64_t>(1, std::min(cells / wa, n[e]));
    wa = std::max<int64_t>(1, std::min(cells / we, n[a]));
    c.lo[a] = (int32_t)(b.lo[a] + (n[a] - wa) / 2);
    c.lo[e] = (int32_t)(b.lo[e] + (n[e] - we) / 2);
    n[a] = wa;
    n[e] = we;
  }
  for (int k = 0; k < 3; ++k) c.n[k] = (int32_t)n[k];
  return c;
}

// The voxel box of a spot extended along the beam's main axis back to the
// face of the grid where the beam enters.  Every proton crosses the air in
// front of the body one voxel per step, close to the spot axis, and each
// crossing deposits: a core window over this extent takes those deposits into
// LDS as well.  An empty box stays empty.
pmc_box to_entry_face(const pmc_box &b, const pmc_field &f, const int n[3]) {
  pmc_box e = b;
  if (b.hi[0] <= b.lo[0] || b.hi[1] <= b.lo[1] || b.hi[2] <= b.lo[2]) return e;
  int d = 0;
  for (int k = 1; k < 3; ++k)
    if (std::fabs(f.direction[k]) > std::fabs(f.direction[d])) d = k;
  if (f.direction[d] < 0.0) e.hi[d] = n[d];
  else e.lo[d] = 0;
  return e;
}

constexpr size_t kMaxPrepared = 32;

// Work items of spots [s0, s1) in queue order.  Each spot's histories are cut
// into runs of `chunk`; the queue holds the first run of every spot (plan
// order), then the second run of every spot that has one, and so on.  Waves
// running at the same time then carry histories of many spots, which spreads
// their tally atomics over many voxels; in plan order every resident wave
// would deposit around the same spot's Bragg peak, and the memory-side atomics
// on those few addresses would serialise.
void build_items(const std::vector<int64_t> &per_spot, int64_t s0, int64_t s1, int64_t chunk,
                 std::vector<WorkItem> &out) {
  std::vector<int32_t> active;
  for (int64_t s = s0; s < s1; ++s)
    if (per_spot[s] > 0) active.push_back((int32_t)s);
  for (int64_t h = 0; !active.empty(); h += chunk) {
    size_t keep = 0;
    for (int32_t s : active) {
      WorkItem w;
      w.spot = s;
      w.h_begin = (uint32_t)h;
      w.h_count = (uint32_t)std::min<int64_t>(chunk, per_spot[s] - h);
      w.pad = 0;
      out.push_back(w);
      if (per_spot[s] > h + chunk) active[keep++] = s;
    }
    active.resize(keep);
  }
}


void evict_lru(pmc_context *ctx) {
  size_t lru = 0;
  for (size_t i = 1; i < ctx->cache.size(); ++i)
    if (ctx->cache[i]->last_use < ctx->cache[lru]->last_use) lru = i;
  wait_use(ctx->cache[lru]->uses);
  drop_use(ctx->cache[lru]->uses);
  release(ctx, ctx->cache[lru]->buf);
  ctx->cache.erase(ctx->cache.begin() + (long)lru);
}

template <typename R>
int build_request(pmc_context *ctx, const pmc_request *req, Prepared &P);

// Split, build and upload the request's device data; cached on the inputs.
template <typename R>
int prepare(pmc_context *ctx, const pmc_request *req, Prepared **out) {
  const PlanRec &plan = ctx->plans[req->plan];
  std::vector<int32_t> phases(req->phases, req->phases + req->n_phases);
  std::vector<uint64_t> versions;
  for (int32_t ph : phases) versions.push_back(ctx->phases[ph].version);
  const LaunchShape shape = launch_shape(ctx, req);
  const int32_t chunk = req->engine == PMC_ENGINE_PERSISTENT ? shape.chunk : 0;
  const int32_t mode = req->engine == PMC_ENGINE_PERSISTENT ? shape.mode : 0;
  for (auto &e : ctx->cache) {
    Prepared &C = *e;
    if (C.plan_id == req->plan && C.plan_version == plan.version && C.n_hist == req->n_histories &&
        C.phases == phases && C.phase_versions == versions && C.engine == req->engine &&
        C.chunk == chunk && C.mode == mode && C.precision == ctx->precision) {
      C.last_use = ++ctx->use_counter;
      *out = &C;
      return PMC_OK;
    }
  }
  auto entry = std::make_unique<Prepared>();
  Prepared &P = *entry;
  int rc = build_request<R>(ctx, req, P);
  if (rc) return rc;
  const size_t off = P.staging.size();
  // room in the cache and in the budget (older entries are evicted first)
  while (!ctx->cache.empty() &&
         (ctx->cache.size() >= kMaxPrepared || ctx->used + align256(off) > ctx->budget))
    evict_lru(ctx);
  rc = ensure(ctx, P.buf, std::max<size_t>(off, 256), "request data");
  if (rc) return rc;
  HIP_TRY(ctx, copy_sync(ctx, P.buf.p, P.staging.data(), off, hipMemcpyHostToDevice),
          "upload request data");
  P.last_use = ++ctx->use_counter;
  ctx->cache.push_back(std::move(entry));
  *out = ctx->cache.back().get();
  return PMC_OK;
}

// The request data of `req` laid out on the host (P.staging, with the
// signature and host-side bookkeeping of P); no device work.
template <typename R>
int build_request(pmc_context *ctx, const pmc_request *req, Prepared &P) {
  const PlanRec &plan = ctx->plans[req->plan];
  std::vector<int32_t> phases(req->phases, req->phases + req->n_phases);
  std::vector<uint64_t> versions;
  for (int32_t ph : phases) versions.push_back(ctx->phases[ph].version);
  const LaunchShape shape = launch_shape(ctx, req);
  const int32_t chunk = req->engine == PMC_ENGINE_PERSISTENT ? shape.chunk : 0;
  const int32_t mode = req->engine == PMC_ENGINE_PERSISTENT ? shape.mode : 0;
  const int64_t n_spots = (int64_t)plan.spots.size();
  P.per_spot.assign(n_spots, 0);
  int rc = split(plan.spots.data(), n_spots, req->phases, req->n_phases, req->n_histories,
                 P.per_spot.data());
  if (rc) return fail(ctx, rc, "history split failed (weights)");
  const int32_t n_slots = req->n_phases;
  std::map<int32_t, int32_t> slot_of;
  for (int32_t i = 0; i < n_slots; ++i) slot_of[phases[i]] = i;
  // spot descriptors
  std::vector<SpotDev<R>> sd(n_spots);
  P.list.assign(n_slots, {});
  P.first.assign(n_slots, {0});
  P.slot_hist.assign(n_slots, 0);
  for (int64_t s = 0; s < n_spots; ++s) {
    const pmc_spot &sp = plan.spots[s];
    auto it = slot_of.find(sp.phase);
    const int32_t slot = it == slot_of.end() ? -1 : it->second;
    const PhaseRec &ph = slot >= 0 ? ctx->phases[sp.phase] : ctx->phases[phases[0]];
    sd[s] = make_spot<R>(sp, plan.fields[sp.field], ph, slot);
    if (slot >= 0 && P.per_spot[s] > 0) {
      P.list[slot].push_back((int32_t)s);
      P.first[slot].push_back(P.first[slot].back() + P.per_spot[s]);
      P.slot_hist[slot] += P.per_spot[s];
      P.incident += (unsigned __int128)((unsigned long long)P.per_spot[s]) *
                    (unsigned long long)q_working(ctx, sp.energy_MeV);
    }
  }
  // work items (persistent engine), in queue order
  std::vector<WorkItem> items;
  if (req->engine == PMC_ENGINE_PERSISTENT) build_items(P.per_spot, 0, n_spots, chunk, items);
  P.n_items = (int32_t)items.size();
  // LUTs: one if all listed phases share it, else one per slot
  const size_t lut_elems = 2 * kLut;
  P.same_lut = true;
  for (int32_t i = 1; i < n_slots; ++i)
    if (ctx->phases[phases[i]].lut64 != ctx->phases[phases[0]].lut64) P.same_lut = false;
  const int32_t n_luts = P.same_lut ? 1 : n_slots;
  // layout of the request data
  size_t off = 0;
  P.off_spots = off;
  off = align256(off + sizeof(SpotDev<R>) * (size_t)n_spots);
  P.off_items = off;
  off = align256(off + sizeof(WorkItem) * items.size());
  // slice cores (block engine), by spot, inside the grid of the spot's phase
  std::vector<pmc::SliceCore> cores;
  if (mode == PMC_TALLY_CORE) {
    P.core_cap = shape.core_cap;
    cores.assign(n_spots, pmc::SliceCore{});
    // a host march along every spot axis, on host threads
    parallel_for(n_spots, [&](int64_t s) {
      const pmc_spot &sp = plan.spots[s];
      if (P.per_spot[s] == 0 || slot_of.find(sp.phase) == slot_of.end()) return;
      cores[s] = slice_core(ctx, ctx->phases.at(sp.phase), plan.fields[sp.field], sp, P.core_cap);
    });
    for (int64_t s = 0; s < n_spots; ++s) {
      const pmc::SliceCore &c = cores[s];
      if (c.n_sl == 0) continue;
      if (c.B[0] != 0 || c.B[1] != 0) P.slanted = true;
      const PhaseRec &ph = ctx->phases.at(plan.spots[s].phase);
      const int n[3] = {ph.nx, ph.ny, ph.nz};
      bool ok = c.d >= 0 && c.d < 3 && c.n_sl > 0 && c.wa > 0 && c.we > 0 &&
                (long long)c.n_sl * c.wa * c.we <= (long long)P.core_cap;
      if (ok) {
        const int a = (c.d + 1) % 3, e = (c.d + 2) % 3;
        ok = c.j0 >= 0 && (long long)c.j0 + c.n_sl <= n[c.d] && c.wa <= n[a] && c.we <= n[e] &&
             c.amin[0] == 0 && c.amin[1] == 0 && c.amax[0] == n[a] - c.wa && c.amax[1] == n[e] - c.we;
        // the corners A + B j in int32 for every slice
        for (int i = 0; i < 2 && ok; ++i) {
          const long long step = (long long)c.B[i] * (c.n_sl - 1);
          ok = std::llabs((long long)c.A[i]) < 2147483647LL && std::llabs(step) < 2147483647LL &&
               std::llabs((long long)c.A[i] + step) < 2147483647LL;
        }
      }
      if (!ok) return fail(ctx, PMC_E_STATE, "internal: slice core of spot %lld out of range", (long long)s);
    }
  }
  P.off_cores = off;
  off = align256(off + sizeof(pmc::SliceCore) * cores.size());
  P.off_luts = off;
  off = align256(off + sizeof(R) * lut_elems * (size_t)n_luts);
  P.off_targets = off;
  off = align256(off + sizeof(TargetDev) * (size_t)n_slots);
  P.off_ids.resize(n_slots);
  P.off_first.resize(n_slots);
  for (int32_t i = 0; i < n_slots; ++i) {
    P.off_ids[i] = off;
    off = align256(off + sizeof(int32_t) * (P.list[i].size() + 1));
    P.off_first[i] = off;
    off = align256(off + sizeof(long long) * P.first[i].size());
  }
  P.staging.assign(off, 0);
  auto put = [&](size_t o, const void *src, size_t n) {
    if (n) std::memcpy(P.staging.data() + o, src, n);
  };
  put(P.off_spots, sd.data(), sizeof(SpotDev<R>) * sd.size());
  put(P.off_items, items.data(), sizeof(WorkItem) * items.size());
  put(P.off_cores, cores.data(), sizeof(pmc::SliceCore) * cores.size());
  for (int32_t l = 0; l < n_luts; ++l) {
    const PhaseRec &ph = ctx->phases[phases[l]];
    const void *src = sizeof(R) == 4 ? (const void *)ph.lut32.data() : (const void *)ph.lut64.data();
    put(P.off_luts + sizeof(R) * lut_elems * l, src, sizeof(R) * lut_elems);
  }
  for (int32_t i = 0; i < n_slots; ++i) {
    put(P.off_ids[i], P.list[i].data(), sizeof(int32_t) * P.list[i].size());
    put(P.off_first[i], P.first[i].data(), sizeof(long long) * P.first[i].size());
  }
  P.bytes = off;
  P.plan_id = req->plan;
  P.plan_version = plan.version;
  P.n_hist = req->n_histories;
  P.phases = phases;
  P.phase_versions = versions;
  P.engine = req->engine;
  P.chunk = chunk;
  P.mode = mode;
  P.precision = ctx->precision;
  return PMC_OK;
}

// Enqueue the transport of a prepared request.  `base` holds the request
// data laid out by prepare() (the context's scratch, or a graph's own copy);
// `cursor` is the work-queue cursor.  With upload_targets false the target
// table at base + off_targets must already hold this call's tally pointers.
// Box tallies of an influence calculation (see pmc_influence).
struct BoxArgs {
  const pmc::BoxDev *boxes;
  unsigned long long *tally;
  long long bias;
  const WorkItem *items;  // the batch's own work items (the spots whose boxes are in tally)
  int32_t n_items;
  const pmc::CoreDev *cores;  // block engine: core window of every spot's box (else null)
  int32_t core_cap;
  const pmc::SliceCore *slices;  // block engine with an oblique field: slice cores instead
};

// Address log of a block-engine launch (pmc_atomic_log).
struct LogArgs {
  unsigned long long *log;
  uint32_t cap;
  uint32_t *count;
};

template <typename R>
int enqueue_prepared(pmc_context *ctx, Prepared &P, const pmc_request *req, hipStream_t st,
                     unsigned long long *const *tally, unsigned long long *counters,
                     unsigned char *base, unsigned long long *cursor, bool upload_targets,
                     const BoxArgs *box = nullptr, unsigned int *drained = nullptr,
                     const LogArgs *log = nullptr) {
  auto scratch_at = [&](size_t off) { return base + off; };
  const bool fp64 = sizeof(R) == 8;
  const uint32_t k0 = (uint32_t)(ctx->seed & 0xffffffffu), k1 = req->request_id;
  const double inv_dl2 = 1.0 / ctx->tabs.dl2;
  if (req->engine == PMC_ENGINE_PLAIN) {
    for (int32_t i = 0; i < req->n_phases; ++i) {
      if (P.slot_hist[i] == 0) continue;
      const PhaseRec &ph = ctx->phases[req->phases[i]];
      pmc::PlainLaunch a;
      a.spots = scratch_at(P.off_spots);
      a.spot_ids = reinterpret_cast<const int32_t *>(scratch_at(P.off_ids[i]));
      a.first = reinterpret_cast<const long long *>(scratch_at(P.off_first[i]));
      a.n_list = (int32_t)P.list[i].size();
      a.n_hist = P.slot_hist[i];
      a.target = make_target(ph, tally[i], 0);
      a.lut = fp64 ? ph.d_lut64 : ph.d_lut32;
      a.tab = ctx->d_tab;
      a.l2e0 = ctx->tabs.l2e0;
      a.inv_dl2 = inv_dl2;
      a.dl2 = ctx->tabs.dl2;
      a.k0 = k0;
      a.k1 = k1;
      a.flags = req->flags;
      a.block = launch_shape(ctx, req).block;
      a.lut_lds = !fp64;
      a.counters = counters;
      HIP_TRY(ctx, pmc::launch_plain(a, fp64, st), "transport_plain launch");
    }
  } else {
    if (upload_targets) {
      // targets carry this call's tally pointers; uploaded only when they
      // change (after the previous user of the table has finished)
      std::vector<TargetDev> tg(req->n_phases);
      for (int32_t i = 0; i < req->n_phases; ++i)
        tg[i] = make_target(ctx->phases[req->phases[i]], tally[i], P.same_lut ? 0 : i);
      const bool same = P.targets.size() == tg.size() &&
                        std::memcmp(P.targets.data(), tg.data(), sizeof(TargetDev) * tg.size()) == 0;
      if (!same) {
        wait_use(P.uses);  // earlier launches of this request read the table
        P.targets = tg;
        HIP_TRY(ctx, copy_sync(ctx, scratch_at(P.off_targets), P.targets.data(),
                               sizeof(TargetDev) * P.targets.size(), hipMemcpyHostToDevice),
                "upload targets");
      }
    }
    HIP_TRY(ctx, pmc::launch_fill_u64(cursor, 1, 0ull, st), "cursor reset");
    pmc::PersistentLaunch a;
    a.spots = scratch_at(P.off_spots);
    // the slice [item_begin, item_end) of the request's work items
    const uint64_t i_end = req->item_end ? req->item_end : (uint64_t)P.n_items;
    a.items = reinterpret_cast<const WorkItem *>(scratch_at(P.off_items)) + req->item_begin;
    a.n_items = (int32_t)(i_end - req->item_begin);
    if (box) {
      a.items = box->items;
      a.n_items = box->n_items;
    }
    a.targets = reinterpret_cast<const TargetDev *>(scratch_at(P.off_targets));
    a.n_targets = req->n_phases;
    a.luts = scratch_at(P.off_luts);
    a.tab = ctx->d_tab;
    a.l2e0 = ctx->tabs.l2e0;
    a.inv_dl2 = inv_dl2;
    a.dl2 = ctx->tabs.dl2;
    a.k0 = k0;
    a.k1 = k1;
    a.flags = req->flags;
    const LaunchShape shape = launch_shape(ctx, req);
    a.refill_min = shape.refill;
    a.block = shape.block;
    if (P.mode == PMC_TALLY_CORE && !box) {
      a.slices = reinterpret_cast<const pmc::SliceCore *>(scratch_at(P.off_cores));
      a.slanted = P.slanted;
      a.core_cap = P.core_cap;
      a.block = pmc::kCoreBlock;
    } else if (box && (box->cores || box->slices)) {
      a.cores = box->cores;
      a.slices = box->slices;
      a.slanted = box->slices != nullptr;
      a.core_cap = box->core_cap;
      a.block = pmc::kCoreBlock;
    }
    a.lut_lds = !fp64 && P.same_lut;
    a.cursor = cursor;
    a.counters = counters;
    if (box) {
      a.boxes = box->boxes;
      a.box_tally = box->tally;
      a.box_bias = box->bias;
    }
    a.drained = drained;
    if (log) {
      if (!a.slices || !a.lut_lds) return fail(ctx, PMC_E_INVAL, "the address log needs the block engine with one LUT");
      a.log = log->log;
      a.log_cap = log->cap;
      a.log_count = log->count;
    }
    unsigned grid = (unsigned)req->grid_blocks;
    if (grid == 0 && (a.cores || a.slices)) {
      // one block per CU (the core takes the LDS), but no more blocks than
      // work items: a block works on one item at a time
      grid = (unsigned)std::max(1, std::min(ctx->n_cu, a.n_items));
    } else if (grid == 0) {
      int per_cu = pmc::persistent_blocks_per_cu(a, fp64);
      if (per_cu < 1) per_cu = 1;
      grid = (unsigned)(ctx->n_cu * per_cu);
      // no more blocks than it takes to start every history of the launch
      // at once (small requests: the others would only stage their tables)
      const uint64_t hist = std::min<uint64_t>(req->n_histories, (uint64_t)a.n_items * (uint64_t)P.chunk);
      const uint64_t need = (hist + (uint64_t)a.block - 1) / (uint64_t)a.block;
      if (need < grid) grid = (unsigned)std::max<uint64_t>(1, need);
    }
    a.grid = grid;
    HIP_TRY(ctx, pmc::launch_persistent(a, fp64, st), "transport_persistent launch");
  }
  return PMC_OK;
}

// One of the context's work-queue cursors for a launch on st: the launch
// that used it before must have finished (a device-side wait on st).  Record
// *done on st after the launch.
int take_cursor(pmc_context *ctx, hipStream_t st, unsigned long long **cursor, hipEvent_t **done) {
  int rc = ensure(ctx, ctx->cursor, 256 * kCursorSlots, "work-queue cursors");
  if (rc) return rc;
  const int slot = ctx->next_cursor;
  ctx->next_cursor = (slot + 1) % kCursorSlots;
  *done = &ctx->cursor_done[slot];
  if (**done) HIP_TRY(ctx, hipStreamWaitEvent(st, **done, 0), "wait for cursor");
  else HIP_TRY(ctx, hipEventCreateWithFlags(*done, hipEventDisableTiming), "hipEventCreate");
  *cursor = reinterpret_cast<unsigned long long *>(static_cast<unsigned char *>(ctx->cursor.p) + 256 * slot);
  return PMC_OK;
}

template <typename R>
int enqueue(pmc_context *ctx, const pmc_request *req, hipStream_t st,
            unsigned long long *const *tally, unsigned long long *counters,
            unsigned int *drained = nullptr, const LogArgs *log = nullptr) {
  Prepared *P = nullptr;
  int rc = prepare<R>(ctx, req, &P);
  if (rc) return rc;
  if (req->item_end > (uint64_t)P->n_items || req->item_begin > (uint64_t)P->n_items)
    return fail(ctx, PMC_E_INVAL, "work-item slice [%llu, %llu) beyond the request's %d items",
                (unsigned long long)req->item_begin, (unsigned long long)req->item_end, P->n_items);
  unsigned long long *cursor = nullptr;
  hipEvent_t *cursor_done = nullptr;
  if (req->engine == PMC_ENGINE_PERSISTENT) {
    rc = take_cursor(ctx, st, &cursor, &cursor_done);
    if (rc) return rc;
  }
  rc = enqueue_prepared<R>(ctx, *P, req, st, tally, counters, static_cast<unsigned char *>(P->buf.p),
                           cursor, true, nullptr, drained, log);
  if (rc) return rc;
  if (cursor_done) HIP_TRY(ctx, hipEventRecord(*cursor_done, st), "hipEventRecord");
  rc = note_use(ctx, P->uses, st);
  for (int32_t i = 0; i < req->n_phases && !rc; ++i) rc = note_use(ctx, ctx->phases[req->phases[i]].uses, st);
  if (rc) return rc;
  return note_pending(ctx, st);
}

// Incident energy of a request (depends only on the split and, for a slice
// of a persistent-engine request, on its work items): 128-bit sum.
int incident_of(pmc_context *ctx, const pmc_request *req, unsigned __int128 *out) {
  const PlanRec &plan = ctx->plans[req->plan];
  std::vector<int64_t> per(plan.spots.size());
  const int rc = split(plan.spots.data(), (int64_t)plan.spots.size(), req->phases, req->n_phases,
                       req->n_histories, per.data());
  if (rc) return fail(ctx, rc, "history split failed");
  unsigned __int128 inc = 0;
  if (req->engine == PMC_ENGINE_PERSISTENT && (req->item_begin || req->item_end)) {
    // the items of the launch (same chunk, same queue order), then the slice
    std::vector<WorkItem> items;
    build_items(per, 0, (int64_t)per.size(), launch_shape(ctx, req).chunk, items);
    const uint64_t e = req->item_end ? std::min<uint64_t>(req->item_end, items.size()) : items.size();
    for (uint64_t k = req->item_begin; k < e; ++k)
      inc += (unsigned __int128)items[k].h_count *
             (unsigned long long)q_working(ctx, plan.spots[items[k].spot].energy_MeV);
  } else {
    for (size_t s = 0; s < per.size(); ++s)
      if (per[s] > 0)
        inc += (unsigned __int128)(unsigned long long)per[s] *
               (unsigned long long)q_working(ctx, plan.spots[s].energy_MeV);
  }
  *out = inc;
  return PMC_OK;
}

void to128(unsigned __int128 v, uint64_t out[2]) {
  out[0] = (uint64_t)v;
  out[1] = (uint64_t)(v >> 64);
}

unsigned __int128 from128(const uint64_t v[2]) {
  return ((unsigned __int128)v[1] << 64) | v[0];
}

void fill_balance(unsigned __int128 incident, const uint64_t *c, unsigned __int128 deposited,
                  pmc_balance *b) {
  to128(incident, b->incident);
  to128(deposited, b->deposited);
  b->escaped[0] = c[0];
  b->escaped[1] = c[1];
  b->nuclear[0] = c[2];
  b->nuclear[1] = c[3];
  b->cutoff[0] = c[4];
  b->cutoff[1] = c[5];
  b->histories = c[6];
  b->steps = c[7];
  b->delta_events = c[8];
  b->nuclear_events = c[9];
  b->escapes = c[10];
  b->misses = c[11];
}

}  // namespace

// ===========================================================================
// exported C ABI
// ===========================================================================
extern "C" {

int pmc_create(const pmc_config *cfg, pmc_context **out) {
  if (!cfg || !out) return fail(nullptr, PMC_E_INVAL, "pmc_create: NULL argument");
  if (cfg->precision != PMC_FP32 && cfg->precision != PMC_FP64)
    return fail(nullptr, PMC_E_INVAL, "precision must be PMC_FP32 or PMC_FP64");
  if (cfg->device < -1) return fail(nullptr, PMC_E_INVAL, "device must be >= -1");
  pmc_context *ctx = new pmc_context();
  ctx->device = cfg->device;
  ctx->precision = cfg->precision;
  ctx->seed = cfg->seed;
  pmc::build_tables(&ctx->tabs);
  if (cfg->device == -1) {  // validation-only context
    ctx->budget = cfg->hbm_budget_bytes ? cfg->hbm_budget_bytes : ~0ull;
    *out = ctx;
    return PMC_OK;
  }
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count <= cfg->device) {
    delete ctx;
    return fail(nullptr, PMC_E_DEVICE, "no HIP device %d (%s)", cfg->device,
                e != hipSuccess ? hipGetErrorString(e) : "device count too small");
  }
  auto bail = [&](hipError_t err, const char *what) {
    const int rc = fail(nullptr, PMC_E_DEVICE, "%s: %s", what, hipGetErrorString(err));
    if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
    if (ctx->d_tab) (void)hipFree(ctx->d_tab);
    delete ctx;
    return rc;
  };
  if ((e = hipSetDevice(cfg->device)) != hipSuccess) return bail(e, "hipSetDevice");
  hipDeviceProp_t prop;
  if ((e = hipGetDeviceProperties(&prop, cfg->device)) != hipSuccess) return bail(e, "hipGetDeviceProperties");
  ctx->n_cu = prop.multiProcessorCount;
  if (prop.sharedMemPerBlock > 0) ctx->lds_max = prop.sharedMemPerBlock;
  size_t free_b = 0, total_b = 0;
  if ((e = hipMemGetInfo(&free_b, &total_b)) != hipSuccess) return bail(e, "hipMemGetInfo");
  ctx->budget = cfg->hbm_budget_bytes ? cfg->hbm_budget_bytes : (uint64_t)(0.9 * (double)free_b);
  if ((e = hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking)) != hipSuccess)
    return bail(e, "hipStreamCreate");
  // the device's scratch for pmc_dose_device_noalloc (first context on the
  // device takes its address; later ones reuse it)
  if ((e = pmc::noalloc_setup(cfg->device, &ctx->noalloc)) != hipSuccess)
    return bail(e, "scratch of the no-allocation entry point");
  // tables in the working precision, per node: (R, mu_delta, omega^2, inverse
  // slope dl2 / (R_{i+1} - R_i) of the interval above the node, 0 at the top)
  const int n = pmc::kTableNodes;
  std::vector<double> islope(n, 0.0);
  for (int i = 0; i + 1 < n; ++i) islope[i] = ctx->tabs.dl2 / (ctx->tabs.range[i + 1] - ctx->tabs.range[i]);
  if (ctx->precision == PMC_FP32) {
    std::vector<float> t(4 * n);
    for (int i = 0; i < n; ++i) {
      t[4 * i + 0] = (float)ctx->tabs.range[i];
      t[4 * i + 1] = (float)ctx->tabs.mu_delta[i];
      t[4 * i + 2] = (float)ctx->tabs.omega2[i];
      t[4 * i + 3] = (float)islope[i];
    }
    ctx->tab_bytes = t.size() * sizeof(float);
    if ((e = hipMalloc(&ctx->d_tab, ctx->tab_bytes)) != hipSuccess) return bail(e, "hipMalloc tables");
    if ((e = hipMemcpy(ctx->d_tab, t.data(), ctx->tab_bytes, hipMemcpyHostToDevice)) != hipSuccess)
      return bail(e, "upload tables");
  } else {
    std::vector<double> t(4 * n);
    for (int i = 0; i < n; ++i) {
      t[4 * i + 0] = ctx->tabs.range[i];
      t[4 * i + 1] = ctx->tabs.mu_delta[i];
      t[4 * i + 2] = ctx->tabs.omega2[i];
      t[4 * i + 3] = islope[i];
    }
    ctx->tab_bytes = t.size() * sizeof(double);
    if ((e = hipMalloc(&ctx->d_tab, ctx->tab_bytes)) != hipSuccess) return bail(e, "hipMalloc tables");
    if ((e = hipMemcpy(ctx->d_tab, t.data(), ctx->tab_bytes, hipMemcpyHostToDevice)) != hipSuccess)
      return bail(e, "upload tables");
  }
  ctx->used = ctx->tab_bytes;
  ctx->has_device = true;
  *out = ctx;
  return PMC_OK;
}

void pmc_destroy(pmc_context *ctx) {
  if (!ctx) return;
  if (ctx->has_device) {
    (void)hipSetDevice(ctx->device);
    wait_pending(ctx);
    wait_noalloc(ctx);
    for (auto &kv : ctx->phases) free_phase(ctx, kv.second);
    for (auto &e : ctx->cache) {
      drop_use(e->uses);
      release(ctx, e->buf);
    }
    ctx->cache.clear();
    release(ctx, ctx->cursor);
    release(ctx, ctx->counters);
    release(ctx, ctx->box_scratch);
    ctx->box_zero = 0;
    release(ctx, ctx->inf_work);
    release(ctx, ctx->inf_rows);
    release(ctx, ctx->inf_voxel);
    release(ctx, ctx->inf_value);
    for (auto &kv : ctx->dvfs) {
      drop_use(kv.second.uses);
      pool_put(ctx, kv.second.d_delta, kv.second.cap);
    }
    ctx->dvfs.clear();
    drop_use(ctx->acc_uses);
    release(ctx, ctx->acc);
    for (hipEvent_t ev : ctx->cursor_done)
      if (ev) (void)hipEventDestroy(ev);
    for (auto &kv : ctx->stream_done) (void)hipEventDestroy(kv.second);
    trim_pool(ctx);
    if (ctx->d_tab) (void)hipFree(ctx->d_tab);
    if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
  }
  delete ctx;
}

const char *pmc_last_error(const pmc_context *ctx) {
  return ctx ? ctx->err.c_str() : g_error.c_str();
}

int pmc_load_phase(pmc_context *ctx, int32_t phase, const int16_t *hu, int32_t nx, int32_t ny,
                   int32_t nz, const double spacing_mm[3], const double origin_mm[3],
                   const double *calib_hu, const double *calib_density, const double *calib_rsp,
                   int32_t n_nodes, const uint8_t *external_mask) {
  if (!ctx) return fail(nullptr, PMC_E_INVAL, "context is NULL");
  ctx->err.clear();
  if (phase < 0 || phase > kMaxPhaseId) return fail(ctx, PMC_E_INVAL, "phase id must be 0..%d", kMaxPhaseId);
  if (!hu || !spacing_mm || !origin_mm || !calib_hu || !calib_density || !calib_rsp)
    return fail(ctx, PMC_E_INVAL, "NULL input array");
  if (nx < 1 || ny < 1 || nz < 1) return fail(ctx, PMC_E_INVAL, "grid dims must be >= 1");
  const long long nvox = (long long)nx * ny * nz;
  if (nvox > 0x7fffffffLL) return fail(ctx, PMC_E_INVAL, "grid has more than 2^31-1 voxels");
  for (int k = 0; k < 3; ++k)
    if (!(std::isfinite(spacing_mm[k]) && spacing_mm[k] > 0.0))
      return fail(ctx, PMC_E_INVAL, "spacing must be finite and > 0");
  if (!finite3(origin_mm)) return fail(ctx, PMC_E_INVAL, "origin must be finite");
  if (n_nodes < 2) return fail(ctx, PMC_E_INVAL, "calibration needs >= 2 nodes");
  for (int i = 0; i < n_nodes; ++i) {
    if (!std::isfinite(calib_hu[i]) || !std::isfinite(calib_density[i]) || !std::isfinite(calib_rsp[i]))
      return fail(ctx, PMC_E_INVAL, "calibration node %d is not finite", i);
    if (calib_density[i] < 0.0 || calib_rsp[i] < 0.0)
      return fail(ctx, PMC_E_INVAL, "calibration node %d has a negative value", i);
    if (i > 0 && !(calib_hu[i] > calib_hu[i - 1]))
      return fail(ctx, PMC_E_INVAL, "calibration HU must be strictly increasing (node %d)", i);
  }
  PhaseRec rec;
  rec.nx = nx;
  rec.ny = ny;
  rec.nz = nz;
  for (int k = 0; k < 3; ++k) {
    rec.sp_mm[k] = spacing_mm[k];
    rec.org_mm[k] = origin_mm[k];
  }
  rec.lut32.resize(2 * kLut);
  rec.lut64.resize(2 * kLut);
  for (int h = kHuLo; h <= kHuHi; ++h) {
    const int i = h - kHuLo;
    const double rho = calib_at(calib_hu, calib_density, n_nodes, (double)h);
    const double rsp = calib_at(calib_hu, calib_rsp, n_nodes, (double)h);
    rec.lut64[2 * i] = rho;
    rec.lut64[2 * i + 1] = rsp;
    rec.lut32[2 * i] = (float)rho;
    rec.lut32[2 * i + 1] = (float)rsp;
  }
  rec.has_mask = external_mask != nullptr;
  rec.hu_host.assign(hu, hu + nvox);
  if (rec.has_mask) rec.mask_host.assign(external_mask, external_mask + nvox);
  rec.version = ++ctx->phase_counter;
  if (!ctx->has_device) {
    auto it = ctx->phases.find(phase);
    if (it != ctx->phases.end()) ctx->phases.erase(it);
    ctx->phases[phase] = std::move(rec);
    return PMC_OK;
  }
  HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  auto cleanup = [&](int rc) {
    free_phase(ctx, rec);
    return rc;
  };
  const size_t l32 = rec.lut32.size() * sizeof(float), l64 = rec.lut64.size() * sizeof(double);
  int rc = pool_get(ctx, (size_t)nvox * 2, (void **)&rec.d_hu, &rec.cap_hu, "phase HU grid");
  if (!rc && rec.has_mask) rc = pool_get(ctx, (size_t)nvox, (void **)&rec.d_mask, &rec.cap_mask, "phase mask");
  if (!rc) rc = pool_get(ctx, l32, &rec.d_lut32, &rec.cap_lut32, "phase LUT");
  if (!rc) rc = pool_get(ctx, l64, &rec.d_lut64, &rec.cap_lut64, "phase LUT");
  if (rc) return cleanup(rc);
  rec.bytes = rec.cap_hu + rec.cap_mask + rec.cap_lut32 + rec.cap_lut64;
  hipError_t e;
  if ((e = copy_sync(ctx, rec.d_hu, hu, (size_t)nvox * 2, hipMemcpyHostToDevice)) != hipSuccess)
    return cleanup(hip_fail(ctx, e, "upload hu"));
  if (rec.has_mask &&
      (e = copy_sync(ctx, rec.d_mask, external_mask, (size_t)nvox, hipMemcpyHostToDevice)) != hipSuccess)
    return cleanup(hip_fail(ctx, e, "upload mask"));
  if ((e = copy_sync(ctx, rec.d_lut32, rec.lut32.data(), l32, hipMemcpyHostToDevice)) != hipSuccess)
    return cleanup(hip_fail(ctx, e, "upload lut"));
  if ((e = copy_sync(ctx, rec.d_lut64, rec.lut64.data(), l64, hipMemcpyHostToDevice)) != hipSuccess)
    return cleanup(hip_fail(ctx, e, "upload lut"));
  auto it = ctx->phases.find(phase);
  if (it != ctx->phases.end()) {
    free_phase(ctx, it->second);
    ctx->phases.erase(it);
  }
  ctx->phases[phase] = std::move(rec);
  return PMC_OK;
}

int pmc_unload_phase(pmc_context *ctx, int32_t phase) {
  if (!ctx) return fail(nullptr, PMC_E_INVAL, "context is NULL");
  ctx->err.clear();
  auto it = ctx->phases.find(phase);
  if (it == ctx->phases.end()) return fail(ctx, PMC_E_NOPHASE, "phase %d is not loaded", phase);
  if (ctx->has_device) {
    (void)hipSetDevice(ctx->device);
    free_phase(ctx, it->second);  // waits for the work that reads it
  }
  ctx->phases.erase(it);
  return PMC_OK;
}

int pmc_load_plan(pmc_context *ctx, int32_t plan, const pmc_field *fields, int32_t n_fields,
                  const pmc_spot *spots, int64_t n_spots) {
  if (!ctx) return fail(nullptr, PMC_E_INVAL, "context is NULL");
  ctx->err.clear();
  if (plan < 0 || plan > kMaxPhaseId) return fail(ctx, PMC_E_INVAL, "plan id must be 0..%d", kMaxPhaseId);
  if (!fields || n_fields < 1) return fail(ctx, PMC_E_INVAL, "need at least one field");
  if (!spots || n_spots < 1 || n_spots > 0x7fffffffLL)
    return fail(ctx, PMC_E_INVAL, "need 1..2^31-1 spots");
  for (int32_t f = 0; f < n_fields; ++f) {
    const pmc_field &F = fields[f];
    if (!finite3(F.isocentre_mm) || !finite3(F.direction) || !finite3(F.bev_u))
      return fail(ctx, PMC_E_INVAL, "field %d: non-finite vector", f);
    const double nd = norm3(F.direction), nu = norm3(F.bev_u);
    const double dot = F.direction[0] * F.bev_u[0] + F.direction[1] * F.bev_u[1] + F.direction[2] * F.bev_u[2];
    if (std::fabs(nd - 1.0) > 1e-6 || std::fabs(nu - 1.0) > 1e-6 || std::fabs(dot) > 1e-6)
      return fail(ctx, PMC_E_INVAL, "field %d: direction and bev_u must be orthogonal unit vectors", f);
  }
  for (int64_t s = 0; s < n_spots; ++s) {
    const pmc_spot &S = spots[s];
    if (!(S.energy_MeV >= PMC_E_MIN_MEV && S.energy_MeV <= PMC_E_MAX_MEV))
      return fail(ctx, PMC_E_INVAL, "spot %lld: energy %g MeV outside [1, 300]", (long long)s, S.energy_MeV);
    if (!std::isfinite(S.x_mm) || !std::isfinite(S.y_mm) || !(S.sigma_mm >= 0.0) || !std::isfinite(S.sigma_mm))
      return fail(ctx, PMC_E_INVAL, "spot %lld: bad position or sigma", (long long)s);
    if (!(S.weight > 0.0) || !std::isfinite(S.weight))
      return fail(ctx, PMC_E_INVAL, "spot %lld: weight must be finite and > 0", (long long)s);
    if (S.field < 0 || S.field >= n_fields)
      return fail(ctx, PMC_E_INVAL, "spot %lld: field %d out of range", (long long)s, S.field);
    if (S.phase < 0 || S.phase > kMaxPhaseId)
      return fail(ctx, PMC_E_INVAL, "spot %lld: phase %d outside 0..%d", (long long)s, S.phase, kMaxPhaseId);
  }
  PlanRec &P = ctx->plans[plan];
  P.fields.assign(fields, fields + n_fields);
  P.spots.assign(spots, spots + n_spots);
  P.version = ++ctx->plan_counter;
  return PMC_OK;
}

int pmc_load_spots(pmc_context *ctx, const pmc_field *fields, int32_t n_fields,
                   const pmc_spot *spots, int64_t n_spots) {
  return pmc_load_plan(ctx, 0, fields, n_fields, spots, n_spots);
}

int pmc_load_subplans(pmc_context *ctx, int32_t plan, const pmc_field *fields, int32_t n_fields,
                      const pmc_spot *spots, int64_t n_spots, const double *mu, int32_t n_phases,
                      const int32_t *phase_ids, int64_t *n_subplan_spots) {
  if (!ctx) return fail(nullptr, PMC_E_INVAL, "context is NULL");
  ctx->err.clear();
  if (!spots || !mu || !phase_ids || n_spots < 1 || n_phases < 1 || n_phases > PMC_MAX_PHASES)
    return fail(ctx, PMC_E_INVAL, "need spots, MU and 1..%d phase ids", PMC_MAX_PHASES);
  for (int32_t p = 0; p < n_phases; ++p)
    if (phase_ids[p] < 0 || phase_ids[p] > kMaxPhaseId)
      return fail(ctx, PMC_E_INVAL, "phase id %d outside 0..%d", phase_ids[p], kMaxPhaseId);
  std::vector<pmc_spot> out;
  for (int64_t s = 0; s < n_spots; ++s)
    for (int32_t p = 0; p < n_phases; ++p) {
      const double m = mu[s * n_phases + p];
      if (!(std::isfinite(m) && m >= 0.0))
        return fail(ctx, PMC_E_INVAL, "MU of spot %lld in phase %d must be finite and >= 0", (long long)s, p);
      if (m > 0.0) {
        pmc_spot sp = spots[s];
        sp.phase = phase_ids[p];
        sp.weight = m;
        out.push_back(sp);
      }
    }
  if (out.empty()) return fail(ctx, PMC_E_INVAL, "no MU delivered: the sub-plans are empty");
  const int rc = pmc_load_plan(ctx, plan, fields, n_fields, out.data(), (int64_t)out.size());
  if (rc == PMC_OK && n_subplan_spots) *n_subplan_spots = (int64_t)out.size();
  return rc;
}

int pmc_unload_plan(pmc_context *ctx, int32_t plan) {
  if (!ctx) return fail(nullptr, PMC_E_INVAL, "context is NULL");
  ctx->err.clear();
  auto it = ctx->plans.find(plan);
  if (it == ctx->plans.end()) return fail(ctx, PMC_E_STATE, "plan %d is not loaded", plan);
  ctx->plans.erase(it);
  // drop the plan's prepared data
  for (size_t i = 0; i < ctx->cache.size();) {
    if (ctx->cache[i]->plan_id == plan) {
      wait_use(ctx->cache[i]->uses);
      drop_use(ctx->cache[i]->uses);
      release(ctx, ctx->cache[i]->buf);
      ctx->cache.erase(ctx->cache.begin() + (long)i);
    } else {
      ++i;
    }
  }
  return PMC_OK;
}

int pmc_request_items(pmc_context *ctx, const pmc_request *req, uint64_t *n_items) {
  if (!ctx) return fail(nullptr, PMC_E_INVAL, "context is NULL");
  ctx->err.clear();
  int rc = validate_request(ctx, req);
  if (rc) return rc;
  if (!n_items) return fail(ctx, PMC_E_INVAL, "n_items is NULL");
  if (req->engine != PMC_ENGINE_PERSISTENT)
    return fail(ctx, PMC_E_INVAL, "work items belong to the persistent engine");
  if (!ctx->has_device) return fail(ctx, PMC_E_DEVICE, "validation-only context has no device");
  HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  Prepared *P = nullptr;
  rc = ctx->precision == PMC_FP64 ? prepare<double>(ctx, req, &P) : prepare<float>(ctx, req, &P);
  if (rc) return rc;
  *n_items = (uint64_t)P->n_items;
  return PMC_OK;
}

int pmc_launch_shape(pmc_context *ctx, const pmc_request *req, pmc_shape *out) {
  if (!ctx) return fail(nullptr, PMC_E_INVAL, "context is NULL");
  ctx->err.clear();
  if (!out) return fail(ctx, PMC_E_INVAL, "out is NULL");
  int rc = validate_request(ctx, req);
  if (rc) return rc;
  const LaunchShape s = launch_shape(ctx, req);
  *out = pmc_shape{};
  out->block_size = s.block;
  out->chunk = s.chunk;
  out->refill_min = s.refill;
  out->tally_mode = s.mode;
  out->core_capacity = s.core_cap;
  return PMC_OK;
}

int pmc_request_item_histories(pmc_context *ctx, const pmc_request *req, uint32_t *histories,
                               uint64_t capacity, uint64_t *n_items) {
  if (!ctx) return fail(nullptr, PMC_E_INVAL, "context is NULL");
  ctx->err.clear();
  int rc = validate_request(ctx, req);
  if (rc) return rc;
  if (req->engine != PMC_ENGINE_PERSISTENT)
    return fail(ctx, PMC_E_INVAL, "work items belong to the persistent engine");
  if (!n_items) return fail(ctx, PMC_E_INVAL, "n_items is NULL");
  const PlanRec &plan = ctx->plans[req->plan];
  const int64_t n_spots = (int64_t)plan.spots.size();
  std::vector<int64_t> per_spot((size_t)n_spots, 0);
  rc = split(plan.spots.data(), n_spots, req->phases, req->n_phases, req->n_histories, per_spot.data());
  if (rc) return fail(ctx, rc, "history split failed (weights)");
  std::vector<WorkItem> items;
  build_items(per_spot, 0, n_spots, default_chunk(ctx, req), items);
  *n_items = (uint64_t)items.size();
  if (!histories) return PMC_OK;
  if (capacity < (uint64_t)items.size())
    return fail(ctx, PMC_E_INVAL, "the request has %zu work items, capacity is %llu", items.size(),
                (unsigned long long)capacity);
  for (size_t i = 0; i < items.size(); ++i) histories[i] = items[i].h_count;
  return PMC_OK;
}

static int dose_device(pmc_context *ctx, const pmc_request *req, void *stream, int64_t *const *dev_tally,
                       uint64_t *dev_counters, unsigned int *drained) {
  if (!ctx) return fail(nullptr, PMC_E_INVAL, "context is NULL");
  ctx->err.clear();
  int rc = validate_request(ctx, req);
  if (rc) return rc;
  if (!dev_tally) return fail(ctx, PMC_E_INVAL, "dev_tally is NULL");
  for (int32_t i = 0; i < req->n_phases; ++i)
    if (!dev_tally[i]) return fail(ctx, PMC_E_INVAL, "dev_tally[%d] is NULL", i);
  if (!ctx->has_device) return fail(ctx, PMC_E_DEVICE, "validation-only context has no device");
  HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  unsigned long long *counters = (unsigned long long *)dev_counters;
  hipStream_t st = (hipStream_t)stream;
  if (!counters) {
    rc = ensure(ctx, ctx->counters, sizeof(uint64_t) * PMC_COUNTERS, "counters");
    if (rc) return rc;
    counters = (unsigned long long *)ctx->counters.p;
    HIP_TRY(ctx, pmc::launch_fill_u64(counters, PMC_COUNTERS, 0ull, st), "counter reset");
  }
  unsigned long long *const *t = reinterpret_cast<unsigned long long *const *>(dev_tally);
  return ctx->precision == PMC_FP64 ? enqueue<double>(ctx, req, st, t, counters, drained)
                                    : enqueue<float>(ctx, req, st, t, counters, drained);
}

int pmc_dose_device(pmc_context *ctx, const pmc_request *req, void *stream,
                    int64_t *const *dev_tally, uint64_t *dev_counters) {
  return dose_device(ctx, req, stream, dev_tally, dev_counters, nullptr);
}

int pmc_dose_device_notify(pmc_context *ctx, const pmc_request *req, void *stream,
                           int64_t *const *dev_tally, uint64_t *dev_counters, uint32_t *host_drained) {
  if (!ctx) return fail(nullptr, PMC_E_INVAL, "context is NULL");
  if (!req || req->engine != PMC_ENGINE_PERSISTENT)
    return fail(ctx, PMC_E_INVAL, "the drain signal belongs to the persistent engine");
  if (!host_drained) return fail(ctx, PMC_E_INVAL, "host_drained is NULL");
  return dose_device(ctx, req, stream, dev_tally, dev_counters, host_drained);
}

int pmc_dose_device_noalloc(pmc_context *ctx, const pmc_request *req, void *stream,
                            int64_t *const *dev_tally, uint64_t *dev_counters) {
  if (!ctx) return fail(nullptr, PMC_E_INVAL, "context is NULL");
  ctx->err.clear();
  int rc = validate_request(ctx, req);
  if (rc) return rc;
  if (!dev_tally) return fail(ctx, PMC_E_INVAL, "dev_tally is NULL");
  for (int32_t i = 0; i < req->n_phases; ++i)
    if (!dev_tally[i]) return fail(ctx, PMC_E_INVAL, "dev_tally[%d] is NULL", i);
  if (!dev_counters) return fail(ctx, PMC_E_INVAL, "dev_counters is NULL (the caller owns the counter block)");
  if (!ctx->has_device || !ctx->noalloc) return fail(ctx, PMC_E_DEVICE, "validation-only context has no device");
  // the request data on the host, laid out as for pmc_dose_device
  Prepared P;
  rc = ctx->precision == PMC_FP64 ? build_request<double>(ctx, req, P) : build_request<float>(ctx, req, P);
  if (rc) return rc;
  if (req->item_end > (uint64_t)P.n_items || req->item_begin > (uint64_t)P.n_items)
    return fail(ctx, PMC_E_INVAL, "work-item slice [%llu, %llu) beyond the request's %d items",
                (unsigned long long)req->item_begin, (unsigned long long)req->item_end, P.n_items);
  const size_t image = align256(P.staging.size());
  const size_t need = image + 256;  // + the work-queue cursor's line
  if (need > pmc::kNoAllocBytes)
    return fail(ctx, PMC_E_RANGE, "request data of %zu bytes exceed the %zu bytes of the no-allocation scratch "
                "(fewer spots or phases, or pmc_dose_device)", need, (size_t)pmc::kNoAllocBytes);
  HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  pmc::NoAlloc &na = *ctx->noalloc;
  // the staging buffer is free once the previous upload from it has ended
  HIP_TRY(ctx, hipEventSynchronize(na.uploaded), "wait for the previous upload");
  std::memcpy(na.host, P.staging.data(), P.staging.size());
  std::vector<TargetDev> tg(req->n_phases);  // this call's tally pointers
  for (int32_t i = 0; i < req->n_phases; ++i)
    tg[i] = make_target(ctx->phases[req->phases[i]], reinterpret_cast<unsigned long long *>(dev_tally[i]),
                        P.same_lut ? 0 : i);
  if (req->engine == PMC_ENGINE_PERSISTENT)
    std::memcpy(na.host + P.off_targets, tg.data(), sizeof(TargetDev) * tg.size());
  HIP_TRY(ctx, hipMemcpyAsync(na.dev, na.host, P.staging.size(), hipMemcpyHostToDevice, st),
          "upload request data");
  HIP_TRY(ctx, hipEventRecord(na.uploaded, st), "hipEventRecord");
  auto *cursor = reinterpret_cast<unsigned long long *>(na.dev + image);
  auto *const *t = reinterpret_cast<unsigned long long *const *>(dev_tally);
  auto *counters = reinterpret_cast<unsigned long long *>(dev_counters);
  ctx->noalloc_used = true;
  return ctx->precision == PMC_FP64
             ? enqueue_prepared<double>(ctx, P, req, st, t, counters, na.dev, cursor, false)
             : enqueue_prepared<float>(ctx, P, req, st, t, counters, na.dev, cursor, false);
}

int pmc_atomic_log(pmc_context *ctx, const pmc_request *req, void *stream, int64_t *const *dev_tally,
                   uint64_t *dev_counters, uint64_t *dev_log, uint32_t per_lane, uint32_t *dev_log_count) {
  if (!ctx) return fail(nullptr, PMC_E_INVAL, "context is NULL");
  ctx->err.clear();
  int rc = validate_request(ctx, req);
  if (rc) return rc;
  if (!dev_tally || !dev_counters || !dev_log || !dev_log_count || per_lane == 0)
    return fail(ctx, PMC_E_INVAL, "NULL tally, counters, log or count, or per_lane = 0");
  for (int32_t i = 0; i < req->n_phases; ++i)
    if (!dev_tally[i]) return fail(ctx, PMC_E_INVAL, "dev_tally[%d] is NULL", i);
  if (req->engine != PMC_ENGINE_PERSISTENT || req->grid_blocks <= 0)
    return fail(ctx, PMC_E_INVAL, "the address log needs the persistent engine and an explicit grid_blocks");
  if (ctx->precision != PMC_FP32) return fail(ctx, PMC_E_INVAL, "the block engine runs in FP32");
  if (launch_shape(ctx, req).mode != PMC_TALLY_CORE)
    return fail(ctx, PMC_E_INVAL, "the request does not run on the block engine (tally_mode)");
  if (!ctx->has_device) return fail(ctx, PMC_E_DEVICE, "validation-only context has no device");
  HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  const LogArgs log{reinterpret_cast<unsigned long long *>(dev_log), per_lane, dev_log_count};
  return enqueue<float>(ctx, req, (hipStream_t)stream, reinterpret_cast<unsigned long long *const *>(dev_tally),
                        reinterpret_cast<unsigned long long *>(dev_counters), nullptr, &log);
}

int pmc_atomic_replay(pmc_context *ctx, void *stream, const uint64_t *dev_log, uint32_t per_lane,
                      const uint32_t *dev_log_count, uint32_t n_lanes) {
  if (!ctx) return fail(nullptr, PMC_E_INVAL, "context is NULL");
  ctx->err.clear();
  if (!dev_log || !dev_log_count || per_lane == 0 || n_lanes == 0 || n_lanes % pmc::kCoreBlock != 0)
    return fail(ctx, PMC_E_INVAL, "NULL log or count, per_lane = 0, or n_lanes not a multiple of %d",
                pmc::kCoreBlock);
  if (!ctx->has_device) return fail(ctx, PMC_E_DEVICE, "validation-only context has no device");
  HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  HIP_TRY(ctx, pmc::launch_atomic_replay(reinterpret_cast<const unsigned long long *>(dev_log), per_lane,
                                         dev_log_count, n_lanes, (hipStream_t)stream),
          "atomic_replay launch");
  return note_pending(ctx, (hipStream_t)stream);
}

int pmc_balance_from_counters(pmc_context *ctx, const pmc_request *req, const uint64_t *counters,
                              const uint64_t deposited[2], pmc_balance *out) {
  if (!ctx) return fail(nullptr, PMC_E_INVAL, "context is NULL");
  ctx->err.clear();
  if (!counters || !deposited || !out) return fail(ctx, PMC_E_INVAL, "NULL argument");
  int rc = validate_request(ctx, req);
  if (rc) return rc;
  unsigned __int128 inc = 0;
  rc = incident_of(ctx, req, &inc);
  if (rc) return rc;
  fill_balance(inc, counters, from128(deposited), out);
  return PMC_OK;
}

int pmc_convert_device(pmc_context *ctx, int32_t phase, const int64_t *dev_tally,
                       uint64_t n_histories, void *stream, double *dev_dose, double *dev_density) {
  if (!ctx) return fail(nullptr, PMC_E_INVAL, "context is NULL");
  ctx->err.clear();
  auto it = ctx->phases.find(phase);
  if (it == ctx->phases.end()) return fail(ctx, PMC_E_NOPHASE, "phase %d is not loaded", phase);
  if (!dev_tally || n_histories == 0) return fail(ctx, PMC_E_INVAL, "need a tally and n_histories >= 1");
  if (!ctx->has_device) return fail(ctx, PMC_E_DEVICE, "validation-only context has no device");
  HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  const PhaseRec &ph = it->second;
  const double vol = (0.1 * ph.sp_mm[0]) * (0.1 * ph.sp_mm[1]) * (0.1 * ph.sp_mm[2]);
  HIP_TRY(ctx, pmc::launch_convert((const long long *)dev_tally, ph.d_hu, ph.d_mask, ph.d_lut64,
                                   ph.nvox(), vol, (double)n_histories, dev_dose, dev_density,
                                   (hipStream_t)stream),
          "convert launch");
  const int rc = note_use(ctx, it->second.uses, (hipStream_t)stream);
  if (rc) return rc;
  return note_pending(ctx, (hipStream_t)stream);
}

int pmc_dose(pmc_context *ctx, const pmc_request *req, double *const *dose_out,
             int64_t *const *tally_out, double *const *density_out, pmc_balance *balance_out) {
  if (!ctx) return fail(nullptr, PMC_E_INVAL, "context is NULL");
  ctx->err.clear();
  int rc = validate_request(ctx, req);
  if (rc) return rc;
  if (!ctx->has_device) return fail(ctx, PMC_E_DEVICE, "validation-only context has no device");
  HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  const int32_t n = req->n_phases;
  // per-call tallies and one dose/density staging buffer
  size_t tally_bytes = 0, max_vox = 0;
  for (int32_t i = 0; i < n; ++i) {
    const long long nv = ctx->phases[req->phases[i]].nvox();
    tally_bytes += (size_t)nv * 8;
    max_vox = std::max(max_vox, (size_t)nv);
  }
  const size_t conv_bytes = max_vox * 8 * 2;
  struct Guard {  // per-call buffers go back to the pool once the call's work is done
    pmc_context *c;
    DevBuf a, b;
    ~Guard() {
      wait_pending(c);
      release(c, a);
      release(c, b);
    }
  } guard{ctx, {}, {}};
  rc = pool_get(ctx, tally_bytes, &guard.a.p, &guard.a.cap, "tallies");
  if (rc) return rc;
  rc = pool_get(ctx, conv_bytes, &guard.b.p, &guard.b.cap, "dose buffer");
  if (rc) return rc;
  void *d_t = guard.a.p, *d_conv = guard.b.p;
  hipStream_t st = ctx->stream;
  HIP_TRY(ctx, hipMemsetAsync(d_t, 0, tally_bytes, st), "zero tallies");
  std::vector<int64_t *> tp(n);
  size_t off = 0;
  for (int32_t i = 0; i < n; ++i) {
    tp[i] = reinterpret_cast<int64_t *>(static_cast<unsigned char *>(d_t) + off);
    off += (size_t)ctx->phases[req->phases[i]].nvox() * 8;
  }
  rc = ensure(ctx, ctx->counters, sizeof(uint64_t) * PMC_COUNTERS, "counters");
  if (rc) return rc;
  HIP_TRY(ctx, hipMemsetAsync(ctx->counters.p, 0, sizeof(uint64_t) * PMC_COUNTERS, st), "zero counters");
  rc = pmc_dose_device(ctx, req, st, tp.data(), (uint64_t *)ctx->counters.p);
  if (rc) return rc;
  // conversion and copies back
  unsigned __int128 deposited = 0;
  std::vector<int64_t> host_tally;
  for (int32_t i = 0; i < n; ++i) {
    const PhaseRec &ph = ctx->phases[req->phases[i]];
    const long long nv = ph.nvox();
    double *d_dose = static_cast<double *>(d_conv);
    double *d_dens = d_dose + nv;
    const bool want_dose = dose_out && dose_out[i];
    const bool want_dens = density_out && density_out[i];
    if (want_dose || want_dens) {
      rc = pmc_convert_device(ctx, req->phases[i], tp[i], req->n_histories, st,
                              want_dose ? d_dose : nullptr, want_dens ? d_dens : nullptr);
      if (rc) return rc;
    }
    int64_t *tdst = (tally_out && tally_out[i]) ? tally_out[i] : nullptr;
    if (!tdst) {
      host_tally.resize((size_t)nv);
      tdst = host_tally.data();
    }
    HIP_TRY(ctx, hipMemcpyAsync(tdst, tp[i], (size_t)nv * 8, hipMemcpyDeviceToHost, st), "copy tally");
    if (want_dose)
      HIP_TRY(ctx, hipMemcpyAsync(dose_out[i], d_dose, (size_t)nv * 8, hipMemcpyDeviceToHost, st), "copy dose");
    if (want_dens)
      HIP_TRY(ctx, hipMemcpyAsync(density_out[i], d_dens, (size_t)nv * 8, hipMemcpyDeviceToHost, st),
              "copy density");
    HIP_TRY(ctx, hipStreamSynchronize(st), "transport / conversion");
    for (long long v = 0; v < nv; ++v) deposited += (unsigned __int128)(uint64_t)tdst[v];
  }
  if (balance_out) {
    uint64_t c[PMC_COUNTERS];
    HIP_TRY(ctx, copy_sync(ctx, c, ctx->counters.p, sizeof c, hipMemcpyDeviceToHost), "copy counters");
    unsigned __int128 inc = 0;
    rc = incident_of(ctx, req, &inc);
    if (rc) return rc;
    fill_balance(inc, c, deposited, balance_out);
  }
  return PMC_OK;
}

int pmc_trace(pmc_context *ctx, int32_t plan, int32_t phase, int64_t spot, uint32_t history,
              uint32_t request_id, uint32_t flags, pmc_trace_rec *out, int32_t max_rec,
              int32_t *n_rec) {
  if (!ctx) return fail(nullptr, PMC_E_INVAL, "context is NULL");
  ctx->err.clear();
  if (!out || max_rec < 1 || !n_rec) return fail(ctx, PMC_E_INVAL, "need an output buffer");
  auto pit = ctx->plans.find(plan);
  if (pit == ctx->plans.end()) return fail(ctx, PMC_E_STATE, "plan %d is not loaded", plan);
  const PlanRec &PL = pit->second;
  if (spot < 0 || spot >= (int64_t)PL.spots.size()) return fail(ctx, PMC_E_INVAL, "spot out of range");
  auto it = ctx->phases.find(phase);
  if (it == ctx->phases.end()) return fail(ctx, PMC_E_NOPHASE, "phase %d is not loaded", phase);
  if (flags & ~31u) return fail(ctx, PMC_E_INVAL, "unknown flag bits");
  if (!ctx->has_device) return fail(ctx, PMC_E_DEVICE, "validation-only context has no device");
  HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  wait_pending(ctx);
  const PhaseRec &ph = it->second;
  const pmc_spot &sp = PL.spots[spot];
  const bool fp64 = ctx->precision == PMC_FP64;
  SpotDev<double> s64 = make_spot<double>(sp, PL.fields[sp.field], ph, 0);
  SpotDev<float> s32 = make_spot<float>(sp, PL.fields[sp.field], ph, 0);
  const size_t rec_bytes = sizeof(pmc_trace_rec) * (size_t)max_rec;
  const size_t tally_bytes = (size_t)ph.nvox() * 8;
  void *d = nullptr;
  HIP_TRY(ctx, hipMalloc(&d, rec_bytes + tally_bytes + 256), "hipMalloc trace");
  struct Free { void *p; ~Free() { (void)hipFree(p); } } fr{d};
  unsigned char *base = static_cast<unsigned char *>(d);
  int32_t *d_n = reinterpret_cast<int32_t *>(base);
  void *d_rec = base + 256;
  void *d_tally = base + 256 + rec_bytes;
  HIP_TRY(ctx, hipMemset(d_tally, 0, tally_bytes), "zero tally");
  pmc::TraceLaunch a;
  a.spot = fp64 ? (const void *)&s64 : (const void *)&s32;
  a.spot_index = (int32_t)spot;
  a.h = history;
  a.target = make_target(ph, (unsigned long long *)d_tally, 0);
  a.lut = fp64 ? ph.d_lut64 : ph.d_lut32;
  a.tab = ctx->d_tab;
  a.l2e0 = ctx->tabs.l2e0;
  a.inv_dl2 = 1.0 / ctx->tabs.dl2;
  a.dl2 = ctx->tabs.dl2;
  a.k0 = (uint32_t)(ctx->seed & 0xffffffffu);
  a.k1 = request_id;
  a.flags = flags;
  a.rec = d_rec;
  a.max_rec = max_rec;
  a.n_rec = d_n;
  HIP_TRY(ctx, pmc::launch_trace(a, fp64, ctx->stream), "trace launch");
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "trace kernel");
  int32_t n = 0;
  HIP_TRY(ctx, copy_sync(ctx, &n, d_n, sizeof n, hipMemcpyDeviceToHost), "copy trace length");
  const int32_t m = std::min(n, max_rec);
  HIP_TRY(ctx, copy_sync(ctx, out, d_rec, sizeof(pmc_trace_rec) * (size_t)m, hipMemcpyDeviceToHost), "copy trace");
  *n_rec = n;
  return PMC_OK;
}

int pmc_split_histories(const pmc_spot *spots, int64_t n_spots, const int32_t *phases,
                        int32_t n_phases, uint64_t n_histories, int64_t *per_spot) {
  if (!spots || n_spots < 1 || !phases || n_phases < 1 || !per_spot)
    return fail(nullptr, PMC_E_INVAL, "pmc_split_histories: bad arguments");
  for (int64_t s = 0; s < n_spots; ++s)
    if (!(spots[s].weight > 0.0) || !std::isfinite(spots[s].weight))
      return fail(nullptr, PMC_E_INVAL, "spot %lld: weight must be finite and > 0", (long long)s);
  const int rc = split(spots, n_spots, phases, n_phases, n_histories, per_spot);
  if (rc) return fail(nullptr, rc, "no spot lies on the listed phases");
  return PMC_OK;
}

uint64_t pmc_bytes_in_use(const pmc_context *ctx) { return ctx ? ctx->used : 0; }

int pmc_graph_create(pmc_context *ctx, const pmc_request *req, int64_t *const *dev_tally,
                     uint64_t *dev_counters, double *const *dev_dose, pmc_graph **out) {
  if (!ctx) return fail(nullptr, PMC_E_INVAL, "context is NULL");
  ctx->err.clear();
  if (!out) return fail(ctx, PMC_E_INVAL, "out is NULL");
  int rc = validate_request(ctx, req);
  if (rc) return rc;
  if (!dev_tally || !dev_counters) return fail(ctx, PMC_E_INVAL, "dev_tally and dev_counters are required");
  for (int32_t i = 0; i < req->n_phases; ++i)
    if (!dev_tally[i]) return fail(ctx, PMC_E_INVAL, "dev_tally[%d] is NULL", i);
  if (!ctx->has_device) return fail(ctx, PMC_E_DEVICE, "validation-only context has no device");
  HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  const bool fp64 = ctx->precision == PMC_FP64;
  Prepared *PP = nullptr;
  rc = fp64 ? prepare<double>(ctx, req, &PP) : prepare<float>(ctx, req, &PP);
  if (rc) return rc;
  if (req->item_end > (uint64_t)PP->n_items || req->item_begin > (uint64_t)PP->n_items)
    return fail(ctx, PMC_E_INVAL, "work-item slice beyond the request's items");
  wait_pending(ctx);
  Prepared &P = *PP;
  const size_t bytes = align256(P.bytes) + 256;  // request data + cursor
  if (ctx->used + bytes > ctx->budget)
    return fail(ctx, PMC_E_BUDGET, "graph data needs %zu bytes: over the device-memory budget", bytes);
  pmc_graph *g = new pmc_graph();
  g->ctx = ctx;
  g->phases.assign(req->phases, req->phases + req->n_phases);
  for (int32_t ph : g->phases) g->versions.push_back(ctx->phases[ph].version);
  g->bytes = bytes;
  auto bail = [&](hipError_t e, const char *what) {
    const int code = hip_fail(ctx, e, what);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->data) { (void)hipFree(g->data); ctx->used -= g->bytes; }
    delete g;
    return code;
  };
  hipError_t e;
  if ((e = hipMalloc(&g->data, bytes)) != hipSuccess) { delete g; return hip_fail(ctx, e, "hipMalloc graph data"); }
  ctx->used += bytes;
  unsigned char *base = static_cast<unsigned char *>(g->data);
  auto *cursor = reinterpret_cast<unsigned long long *>(base + align256(P.bytes));
  // private image of the request data with this graph's tally pointers
  std::vector<unsigned char> image = P.staging;
  std::vector<TargetDev> tg(req->n_phases);
  for (int32_t i = 0; i < req->n_phases; ++i)
    tg[i] = make_target(ctx->phases[req->phases[i]], reinterpret_cast<unsigned long long *>(dev_tally[i]),
                        P.same_lut ? 0 : i);
  std::memcpy(image.data() + P.off_targets, tg.data(), sizeof(TargetDev) * tg.size());
  if ((e = copy_sync(ctx, base, image.data(), P.bytes, hipMemcpyHostToDevice)) != hipSuccess)
    return bail(e, "upload graph data");
  hipStream_t st = ctx->stream;
  if ((e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal)) != hipSuccess)
    return bail(e, "hipStreamBeginCapture");
  auto *counters = reinterpret_cast<unsigned long long *>(dev_counters);
  bool ok = true;
  for (int32_t i = 0; i < req->n_phases && ok; ++i)
    ok = pmc::launch_fill_u64(reinterpret_cast<unsigned long long *>(dev_tally[i]),
                              ctx->phases[req->phases[i]].nvox(), 0ull, st) == hipSuccess;
  ok = ok && pmc::launch_fill_u64(counters, PMC_COUNTERS, 0ull, st) == hipSuccess;
  auto *const *tp = reinterpret_cast<unsigned long long *const *>(dev_tally);
  if (ok)
    rc = fp64 ? enqueue_prepared<double>(ctx, P, req, st, tp, counters, base, cursor, false)
              : enqueue_prepared<float>(ctx, P, req, st, tp, counters, base, cursor, false);
  ok = ok && rc == PMC_OK;
  for (int32_t i = 0; i < req->n_phases && ok && dev_dose; ++i) {
    if (!dev_dose[i]) continue;
    const PhaseRec &ph = ctx->phases[req->phases[i]];
    const double vol = (0.1 * ph.sp_mm[0]) * (0.1 * ph.sp_mm[1]) * (0.1 * ph.sp_mm[2]);
    ok = pmc::launch_convert(reinterpret_cast<const long long *>(dev_tally[i]), ph.d_hu, ph.d_mask,
                             ph.d_lut64, ph.nvox(), vol, (double)req->n_histories, dev_dose[i],
                             nullptr, st) == hipSuccess;
  }
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(st, &graph);
  g->graph = graph;
  if (!ok) {
    const std::string msg = ctx->err.empty() ? "launch failed during capture" : ctx->err;
    bail(hipErrorUnknown, "graph capture");
    return fail(ctx, rc ? rc : PMC_E_DEVICE, "graph capture: %s", msg.c_str());
  }
  if (e != hipSuccess) return bail(e, "hipStreamEndCapture");
  if ((e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0)) != hipSuccess)
    return bail(e, "hipGraphInstantiate");
  *out = g;
  return PMC_OK;
}

int pmc_graph_launch(pmc_graph *g, void *stream) {
  if (!g) return fail(nullptr, PMC_E_INVAL, "graph is NULL");
  pmc_context *ctx = g->ctx;
  ctx->err.clear();
  // the captured kernels read the phases' HU grids, masks and LUTs by
  // address: a phase unloaded or replaced since the capture has returned
  // that memory to the pool, so the graph must not run
  for (size_t i = 0; i < g->phases.size(); ++i) {
    auto it = ctx->phases.find(g->phases[i]);
    if (it == ctx->phases.end() || it->second.version != g->versions[i])
      return fail(ctx, PMC_E_STATE, "phase %d was unloaded or replaced since the graph was captured",
                  g->phases[i]);
  }
  HIP_TRY(ctx, hipGraphLaunch(g->exec, (hipStream_t)stream), "hipGraphLaunch");
  for (int32_t ph : g->phases) {
    const int rc = note_use(ctx, ctx->phases[ph].uses, (hipStream_t)stream);
    if (rc) return rc;
  }
  return note_pending(ctx, (hipStream_t)stream);
}

void pmc_graph_destroy(pmc_graph *g) {
  if (!g) return;
  (void)hipSetDevice(g->ctx->device);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->data) {
    (void)hipDeviceSynchronize();
    (void)hipFree(g->data);
    g->ctx->used -= g->bytes;
  }
  delete g;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// influence matrix
// ---------------------------------------------------------------------------
namespace {

// Restricted CSDA range in water (g/cm^2) at E, from the transport tables.
double table_range(const pmc::Tables &T, double E) {
  double x = (std::log2(E) - T.l2e0) / T.dl2;
  int i = (int)x;
  i = i < 0 ? 0 : (i > pmc::kTableNodes - 2 ? pmc::kTableNodes - 2 : i);
  const double f = x - i;
  return T.range[i] + f * (T.range[i + 1] - T.range[i]);
}

double rsp_at(const PhaseRec &ph, long long v) {
  if (ph.has_mask && ph.mask_host[(size_t)v] == 0) return 0.0;
  int h = ph.hu_host[(size_t)v];
  h = h < kHuLo ? kHuLo : (h > kHuHi ? kHuHi : h);
  return ph.lut64[2 * (h - kHuLo) + 1];
}

// Voxel box of a spot: the spot's central axis from where it first meets
// matter (stopping-power ratio >= kBodyRsp; air before it is left out) to
// water-equivalent depth R(E) + 3 cm (or the grid exit), widened by
// 3 sigma_max across the beam, sigma_max^2 = sigma_spot^2 + (0.035 L)^2 with
// L the geometric length of that axis segment.
constexpr double kBodyRsp = 0.1;

// The central axis of a spot in grid coordinates (cm from the grid corner):
// c + t w, BEV axes u and v, voxel size d; [t_in, t_out) inside the grid
// box; t_body where it first meets matter, t_end at water-equivalent depth
// R(E) + margin_cm (or the grid exit).  False if the axis misses the grid or
// meets no matter.
struct AxisRay {
  double w[3], u[3], v[3], c[3], d[3];
  int n[3];
  double t_in, t_out, t_body, t_end;
};

bool axis_ray(const pmc_context *ctx, const PhaseRec &ph, const pmc_field &f, const pmc_spot &s,
              double margin_cm, AxisRay &A) {
  double *w = A.w, *u = A.u, *v = A.v, *c = A.c, *d = A.d;
  double ext[3];
  int *n = A.n;
  n[0] = ph.nx;
  n[1] = ph.ny;
  n[2] = ph.nz;
  const double nw = norm3(f.direction), nu = norm3(f.bev_u);
  for (int k = 0; k < 3; ++k) {
    w[k] = f.direction[k] / nw;
    u[k] = f.bev_u[k] / nu;
  }
  v[0] = w[1] * u[2] - w[2] * u[1];
  v[1] = w[2] * u[0] - w[0] * u[2];
  v[2] = w[0] * u[1] - w[1] * u[0];
  for (int k = 0; k < 3; ++k) {
    c[k] = 0.1 * (f.isocentre_mm[k] - ph.org_mm[k]) + 0.1 * s.x_mm * u[k] + 0.1 * s.y_mm * v[k];
    d[k] = 0.1 * ph.sp_mm[k];
    ext[k] = n[k] * d[k];
  }
  double t_in = -HUGE_VAL, t_out = HUGE_VAL;
  for (int k = 0; k < 3; ++k) {
    if (w[k] != 0.0) {
      const double t1 = (0.0 - c[k]) / w[k], t2 = (ext[k] - c[k]) / w[k];
      t_in = std::max(t_in, std::min(t1, t2));
      t_out = std::min(t_out, std::max(t1, t2));
    } else if (c[k] < 0.0 || c[k] >= ext[k]) {
      return false;
    }
  }
  if (!(t_in < t_out)) return false;
  // march the axis through the voxels, accumulating water-equivalent depth
  const double target = table_range(ctx->tabs, s.energy_MeV) + margin_cm;
  int idx[3];
  double t_max[3], t_step[3];
  const double tm = 0.5 * (t_in + std::min(t_out, t_in + 1e-6));
  for (int k = 0; k < 3; ++k) {
    const double p = c[k] + tm * w[k];
    idx[k] = std::min(n[k] - 1, std::max(0, (int)std::floor(p / d[k])));
    if (w[k] > 0.0) { t_max[k] = ((idx[k] + 1) * d[k] - c[k]) / w[k]; t_step[k] = d[k] / w[k]; }
    else if (w[k] < 0.0) { t_max[k] = (idx[k] * d[k] - c[k]) / w[k]; t_step[k] = -d[k] / w[k]; }
    else { t_max[k] = HUGE_VAL; t_step[k] = HUGE_VAL; }
  }
  double t = t_in, wet = 0.0, t_end = t_out, t_body = -HUGE_VAL;
  for (;;) {
    int ax = 0;
    if (t_max[1] < t_max[ax]) ax = 1;
    if (t_max[2] < t_max[ax]) ax = 2;
    const double t_next = std::min(t_max[ax], t_out);
    const long long vx = (long long)idx[0] + (long long)n[0] * ((long long)idx[1] + (long long)n[1] * idx[2]);
    const double r = rsp_at(ph, vx);
    if (t_body == -HUGE_VAL && r >= kBodyRsp) t_body = t;
    const double seg = std::max(0.0, t_next - t);
    if (r > 0.0 && wet + r * seg >= target) {
      t_end = t + (target - wet) / r;
      break;
    }
    wet += r * seg;
    t = t_next;
    if (t >= t_out) break;
    idx[ax] += w[ax] > 0.0 ? 1 : -1;
    if (idx[ax] < 0 || idx[ax] >= n[ax]) break;
    t_max[ax] += t_step[ax];
  }
  if (t_body == -HUGE_VAL) return false;  // no matter on the axis
  A.t_in = t_in;
  A.t_out = t_out;
  A.t_body = t_body;
  A.t_end = t_end;
  return true;
}

pmc_box spot_box(const pmc_context *ctx, const PhaseRec &ph, const pmc_field &f, const pmc_spot &s) {
  pmc_box b = {{0, 0, 0}, {0, 0, 0}};
  AxisRay A;
  if (!axis_ray(ctx, ph, f, s, 3.0, A)) return b;
  const double L = A.t_end - A.t_body;
  const double sig = 0.1 * s.sigma_mm;
  const double r = 3.0 * std::sqrt(sig * sig + (0.035 * L) * (0.035 * L));
  for (int k = 0; k < 3; ++k) {
    const double a = A.c[k] + A.t_body * A.w[k], e = A.c[k] + A.t_end * A.w[k];
    const double half = r * (std::fabs(A.u[k]) + std::fabs(A.v[k]));
    const double lo = std::min(a, e) - half, hi = std::max(a, e) + half;
    long long il = (long long)std::floor(lo / A.d[k]), ih = (long long)std::floor(hi / A.d[k]) + 1;
    il = std::max(0LL, std::min((long long)A.n[k], il));
    ih = std::max(0LL, std::min((long long)A.n[k], ih));
    b.lo[k] = (int32_t)il;
    b.hi[k] = (int32_t)ih;
  }
  for (int k = 0; k < 3; ++k)
    if (b.hi[k] <= b.lo[k]) return pmc_box{{0, 0, 0}, {0, 0, 0}};
  return b;
}

// Block-engine core of a spot (pmc::SliceCore).  The slices are those of
// the grid axis d closest to the beam, from the face where the axis enters
// the grid to the slice where it reaches water-equivalent depth R(E) + 1 cm
// (beyond it the protons have stopped); each holds a window of the same
// wa x we voxels across, centred on the axis at the slice's middle plane and
// clamped into the grid, so that the core follows an oblique beam.  The
// window's aspect ratio is that of the beam's cross-section cut by a slice.
// With `inside` (influence calculations) slices and windows are kept inside
// that box.  n_sl wa we <= cap; no core (n_sl = 0) when the axis misses the
// grid or the box, meets no matter, or the slices alone exceed cap.
pmc::SliceCore slice_core(const pmc_context *ctx, const PhaseRec &ph, const pmc_field &f, const pmc_spot &s,
                          int32_t cap, const pmc_box *inside) {
  pmc::SliceCore sc = {};
  AxisRay A;
  if (cap <= 0 || !axis_ray(ctx, ph, f, s, 1.0, A)) return sc;
  int rlo[3] = {0, 0, 0}, rhi[3] = {A.n[0], A.n[1], A.n[2]};
  if (inside) {
    for (int k = 0; k < 3; ++k) {
      rlo[k] = std::max(0, inside->lo[k]);
      rhi[k] = std::min(A.n[k], inside->hi[k]);
      if (rhi[k] <= rlo[k]) return sc;
    }
  }
  int d = 0;
  for (int k = 1; k < 3; ++k)
    if (std::fabs(A.w[k]) > std::fabs(A.w[d])) d = k;
  const int a = (d + 1) % 3, e = (d + 2) % 3;
  auto slice_at = [&](double t) {
    const long long j = (long long)std::floor((A.c[d] + t * A.w[d]) / A.d[d]);
    return std::max(0LL, std::min((long long)A.n[d] - 1, j));
  };
  // the entry slice: just inside the grid (t_in is on its face)
  const long long j_in = slice_at(A.t_in + 1e-9 * (A.t_out - A.t_in)), j_end = slice_at(A.t_end);
  const long long j0 = std::max((long long)rlo[d], std::min(j_in, j_end));
  const long long j1 = std::min((long long)rhi[d] - 1, std::max(j_in, j_end));
  if (j1 < j0) return sc;
  const long long n_sl = j1 - j0 + 1;
  if (n_sl > cap || n_sl > (1 << 15)) return sc;
  const long long cells = cap / n_sl;
  // cross-section of the beam in a slice: a lateral offset r (along u or v)
  // moves the crossing point by r (u_k - u_d w_k / w_d) along axis k
  auto foot = [&](int k) {
    const double p = A.u[k] - A.u[d] * A.w[k] / A.w[d], q = A.v[k] - A.v[d] * A.w[k] / A.w[d];
    return std::max(1e-3, std::sqrt(p * p + q * q)) / A.d[k];
  };
  const long long na = rhi[a] - rlo[a], ne = rhi[e] - rlo[e];
  long long wa = (long long)std::floor(std::sqrt((double)cells * foot(a) / foot(e)));
  wa = std::max(1LL, std::min(wa, na));
  long long we = std::max(1LL, std::min(cells / wa, ne));
  wa = std::max(1LL, std::min(cells / we, na));
  // window corner along k at slice j: the axis at the slice's middle plane
  // minus half the width, in 16.16 fixed point, linear in j
  const int ax[2] = {a, e};
  const long long wid[2] = {wa, we};
  for (int i = 0; i < 2; ++i) {
    const int k = ax[i];
    const double slope = A.w[k] * A.d[d] / (A.w[d] * A.d[k]);  // voxels along k per slice
    const double t0 = ((double)j0 + 0.5) * A.d[d] - A.c[d];
    const double first = (A.c[k] + t0 / A.w[d] * A.w[k]) / A.d[k] - 0.5 * (double)wid[i] + 0.5;
    const double fa = std::floor(first * 65536.0), fb = std::floor(slope * 65536.0 + 0.5);
    // every corner A + B j of the slices in int32
    const double lim = 2147483647.0 - 65536.0;
    if (!(std::fabs(fa) < lim && std::fabs(fb * (double)(n_sl - 1)) < lim &&
          std::fabs(fa + fb * (double)(n_sl - 1)) < lim))
      return pmc::SliceCore{};
    sc.A[i] = (int32_t)fa;
    sc.B[i] = (int32_t)fb;
    sc.amin[i] = rlo[k];
    sc.amax[i] = (int32_t)(rhi[k] - wid[i]);
  }
  sc.d = d;
  sc.j0 = (int32_t)j0;
  sc.n_sl = (int32_t)n_sl;
  sc.wa = (int32_t)wa;
  sc.we = (int32_t)we;
  return sc;
}

long long box_entries(const pmc_box &b) {
  long long e = 1;
  for (int k = 0; k < 3; ++k) e *= (long long)(b.hi[k] - b.lo[k]);
  return e;
}

int grow_csr(pmc_context *ctx, size_t need, hipStream_t st) {
  if (need <= ctx->inf_cap) return PMC_OK;
  const size_t cap = std::max(need, ctx->inf_cap + ctx->inf_cap / 2);
  const size_t add = (cap - ctx->inf_cap) * (sizeof(int32_t) + sizeof(float));
  if (ctx->used + add > ctx->budget)
    return fail(ctx, PMC_E_BUDGET, "influence matrix: %zu entries exceed the device-memory budget", cap);
  void *nv = nullptr, *nf = nullptr;
  HIP_TRY(ctx, hipMalloc(&nv, cap * sizeof(int32_t)), "hipMalloc influence voxels");
  if (hipMalloc(&nf, cap * sizeof(float)) != hipSuccess) {
    (void)hipFree(nv);
    return fail(ctx, PMC_E_DEVICE, "hipMalloc influence values");
  }
  if (ctx->inf_nnz) {
    HIP_TRY(ctx, hipMemcpyAsync(nv, ctx->inf_voxel.p, ctx->inf_nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, st),
            "copy influence voxels");
    HIP_TRY(ctx, hipMemcpyAsync(nf, ctx->inf_value.p, ctx->inf_nnz * sizeof(float), hipMemcpyDeviceToDevice, st),
            "copy influence values");
  }
  HIP_TRY(ctx, hipStreamSynchronize(st), "influence copy");
  release(ctx, ctx->inf_voxel);
  release(ctx, ctx->inf_value);
  ctx->inf_voxel.p = nv;
  ctx->inf_voxel.cap = cap * sizeof(int32_t);
  ctx->inf_value.p = nf;
  ctx->inf_value.cap = cap * sizeof(float);
  ctx->used += cap * (sizeof(int32_t) + sizeof(float));
  ctx->inf_cap = cap;
  return PMC_OK;
}

void free_influence(pmc_context *ctx) {
  release(ctx, ctx->box_scratch);
  ctx->box_zero = 0;
  release(ctx, ctx->inf_work);
  release(ctx, ctx->inf_rows);
  release(ctx, ctx->inf_voxel);
  release(ctx, ctx->inf_value);
  ctx->inf_cap = 0;
  ctx->inf_nnz = 0;
  ctx->inf_n_rows = -1;
}

template <typename R>
int influence(pmc_context *ctx, const pmc_request *req_in, const pmc_box *boxes_in, double thr,
              uint64_t max_scratch, uint64_t *nnz_out, pmc_balance *bal_out, uint64_t outside_out[2]) {
  pmc_request rq = *req_in;
  rq.engine = PMC_ENGINE_PERSISTENT;
  rq.tally_mode = PMC_TALLY_LANE;  // per-spot box tallies
  const PlanRec &plan = ctx->plans[rq.plan];
  const int64_t n_spots = (int64_t)plan.spots.size();
  const int32_t phase_id = rq.phases[0];
  const PhaseRec &ph = ctx->phases[phase_id];
  // boxes
  std::vector<pmc_box> bx((size_t)n_spots, pmc_box{{0, 0, 0}, {0, 0, 0}});
  if (boxes_in) {
    for (int64_t s = 0; s < n_spots; ++s) {
      bx[s] = boxes_in[s];
      const int n[3] = {ph.nx, ph.ny, ph.nz};
      for (int k = 0; k < 3; ++k)
        if (bx[s].lo[k] < 0 || bx[s].hi[k] > n[k] || bx[s].lo[k] > bx[s].hi[k])
          return fail(ctx, PMC_E_INVAL, "box of spot %lld is not inside the grid", (long long)s);
    }
  } else {
    parallel_for(n_spots, [&](int64_t s) {
      if (plan.spots[s].phase == phase_id)
        bx[s] = spot_box(ctx, ph, plan.fields[plan.spots[s].field], plan.spots[s]);
    });
  }
  Prepared *P = nullptr;
  int rc = prepare<R>(ctx, &rq, &P);
  if (rc) return rc;
  const int64_t chunk = P->chunk;
  // device boxes, tile layout and the work-item range of every spot
  std::vector<pmc::BoxDev> bd((size_t)n_spots);
  std::vector<long long> offset((size_t)n_spots + 1, 0);
  long long largest = 0;
  for (int64_t s = 0; s < n_spots; ++s) {
    pmc::BoxDev &d = bd[s];
    const int64_t h = P->per_spot[s];
    const long long ne = h > 0 ? box_entries(bx[s]) : 0;
    if (ne > (1LL << 31) - 2 * pmc::kTile)
      return fail(ctx, PMC_E_INVAL, "box of spot %lld has more than 2^31 - 2048 voxels", (long long)s);
    for (int k = 0; k < 3; ++k) {
      d.lo[k] = bx[s].lo[k];
      d.n[k] = ne > 0 ? bx[s].hi[k] - bx[s].lo[k] : 0;
    }
    d.offset = offset[s];
    d.n_hist = (double)h;
    d.pad = 0.0;
    const long long padded = (ne + pmc::kTile - 1) / pmc::kTile * pmc::kTile;
    largest = std::max(largest, padded);
    offset[s + 1] = offset[s] + padded;
  }
  // batches of consecutive spots whose boxes fit the scratch
  const size_t free_b = ctx->budget > ctx->used ? ctx->budget - ctx->used : 0;
  const size_t scratch_b = max_scratch ? std::min<size_t>(max_scratch, free_b) : free_b / 2;
  if ((size_t)largest * sizeof(long long) > scratch_b)
    return fail(ctx, PMC_E_BUDGET, "a spot box of %lld voxels exceeds the scratch allowed (%zu bytes)",
                largest, scratch_b);
  const long long cap = (long long)(scratch_b / sizeof(long long));
  std::vector<int64_t> cuts = {0};
  for (int64_t s = 0; s < n_spots; ++s)
    if (offset[s + 1] - offset[cuts.back()] > cap) cuts.push_back(s);
  cuts.push_back(n_spots);
  long long max_entries = 0, max_spots = 0;
  for (size_t b = 0; b + 1 < cuts.size(); ++b) {
    max_entries = std::max(max_entries, offset[cuts[b + 1]] - offset[cuts[b]]);
    max_spots = std::max<long long>(max_spots, cuts[b + 1] - cuts[b]);
  }
  const long long max_tiles = max_entries / pmc::kTile, max_chunks = (max_tiles + 1023) / 1024;
  // Block engine (FP32, room in LDS, items of kCoreChunk averaging one
  // history per lane, as for dense requests): every spot's box keeps a core
  // window in LDS.  Else the lane engine with the request's chunk.
  // The request's tally_mode forces either engine.
  int32_t core_cap = 0;
  int64_t item_chunk = chunk;
  if (ctx->precision == PMC_FP32 && req_in->tally_mode != PMC_TALLY_LANE) {
    const int32_t cap = core_capacity(ctx, P->same_lut);
    const int64_t core_chunk = req_in->chunk > 0 ? req_in->chunk : kCoreChunk;
    int64_t items = 0;
    for (int64_t h : P->per_spot) items += (h + core_chunk - 1) / core_chunk;
    const int64_t n_cu = ctx->n_cu > 0 ? ctx->n_cu : 256;
    const bool pick = req_in->tally_mode == PMC_TALLY_CORE ||
                      (cap >= kCoreMinEntries && (int64_t)rq.n_histories >= (int64_t)pmc::kCoreBlock * items &&
                       (int64_t)rq.n_histories >= (int64_t)pmc::kCoreBlock * n_cu);
    if (pick && cap > 0) {
      core_cap = cap;
      item_chunk = core_chunk;
    }
  }
  // the core of every spot: when some field runs oblique to the grid, slice
  // cores inside the boxes (windows that follow the beam axis); else a
  // window of each box
  std::vector<pmc::CoreDev> cores;
  std::vector<pmc::SliceCore> slices;
  bool slanted = false;
  if (core_cap > 0) {
    slices.assign((size_t)n_spots, pmc::SliceCore{});
    parallel_for(n_spots, [&](int64_t s) {
      if (P->per_spot[s] == 0) return;
      const pmc_spot &sp = plan.spots[s];
      slices[s] = slice_core(ctx, ph, plan.fields[sp.field], sp, core_cap, &bx[s]);
    });
    for (int64_t s = 0; s < n_spots; ++s) {
      const pmc::SliceCore &c = slices[s];
      if (c.n_sl == 0) continue;
      if (c.B[0] != 0 || c.B[1] != 0) slanted = true;
      bool ok = c.d >= 0 && c.d < 3 && c.wa > 0 && c.we > 0 &&
                (long long)c.n_sl * c.wa * c.we <= (long long)core_cap;
      if (ok) {
        const int a = (c.d + 1) % 3, e = (c.d + 2) % 3;
        ok = c.j0 >= bx[s].lo[c.d] && c.j0 + c.n_sl <= bx[s].hi[c.d] && c.amin[0] == bx[s].lo[a] &&
             c.amin[1] == bx[s].lo[e] && c.amax[0] == bx[s].hi[a] - c.wa && c.amax[1] == bx[s].hi[e] - c.we &&
             c.amax[0] >= c.amin[0] && c.amax[1] >= c.amin[1];
        for (int i = 0; i < 2 && ok; ++i) {
          const long long step = (long long)c.B[i] * (c.n_sl - 1);
          ok = std::llabs((long long)c.A[i]) < 2147483647LL && std::llabs(step) < 2147483647LL &&
               std::llabs((long long)c.A[i] + step) < 2147483647LL;
        }
      }
      if (!ok) return fail(ctx, PMC_E_STATE, "internal: slice core of spot %lld outside its box", (long long)s);
    }
    if (!slanted) {
      slices.clear();
      cores.assign((size_t)n_spots, pmc::CoreDev{});
      for (int64_t s = 0; s < n_spots; ++s) {
        if (P->per_spot[s] == 0) continue;
        pmc::CoreDev c = core_of(bx[s], plan.fields[plan.spots[s].field], core_cap);
        bool ok = (long long)c.n[0] * c.n[1] * c.n[2] <= (long long)core_cap;
        for (int k = 0; k < 3; ++k)
          ok = ok && c.n[k] >= 0 && c.lo[k] >= bx[s].lo[k] && c.lo[k] + c.n[k] <= bx[s].hi[k];
        if (!ok) return fail(ctx, PMC_E_STATE, "internal: core window of spot %lld outside its box", (long long)s);
        cores[s] = c;
      }
    }
  }
  // each batch's work items, in queue order over its spots
  std::vector<WorkItem> bitems;
  std::vector<size_t> batch_first = {0};
  for (size_t b = 0; b + 1 < cuts.size(); ++b) {
    build_items(P->per_spot, cuts[b], cuts[b + 1], item_chunk, bitems);
    batch_first.push_back(bitems.size());
  }
  // work buffer layout
  size_t off = 0;
  const size_t o_boxes = off; off = align256(off + sizeof(pmc::BoxDev) * (size_t)n_spots);
  const size_t o_tfirst = off; off = align256(off + sizeof(long long) * (size_t)(max_spots + 1));
  const size_t o_max = off; off = align256(off + sizeof(long long) * (size_t)max_spots);
  const size_t o_dep = off; off = align256(off + 2 * sizeof(long long));
  const size_t o_count = off; off = align256(off + 2 * sizeof(uint32_t) * (size_t)max_tiles);  // count, keep
  const size_t o_toff = off; off = align256(off + sizeof(long long) * (size_t)max_tiles);
  const size_t o_coff = off; off = align256(off + sizeof(long long) * (size_t)(max_chunks + 1));
  const size_t o_items = off; off = align256(off + sizeof(WorkItem) * bitems.size());
  const size_t o_cores = off;
  off = align256(off + std::max(sizeof(pmc::CoreDev) * cores.size(), sizeof(pmc::SliceCore) * slices.size()));
  ctx->inf_n_rows = -1;
  ctx->inf_nnz = 0;
  rc = ensure(ctx, ctx->inf_work, std::max<size_t>(off, 256), "influence work buffer");
  if (rc) return rc;
  void *const old_scratch = ctx->box_scratch.p;
  rc = ensure(ctx, ctx->box_scratch, std::max<size_t>((size_t)max_entries * sizeof(long long), 256),
              "influence box tallies");
  if (rc) return rc;
  if (ctx->box_scratch.p != old_scratch) ctx->box_zero = 0;  // memory of the pool: contents unknown
  rc = ensure(ctx, ctx->inf_rows, sizeof(int64_t) * (size_t)(n_spots + 1), "influence rows");
  if (rc) return rc;
  rc = ensure(ctx, ctx->counters, sizeof(uint64_t) * PMC_COUNTERS, "counters");
  if (rc) return rc;
  unsigned char *work = static_cast<unsigned char *>(ctx->inf_work.p);
  auto *d_boxes = reinterpret_cast<pmc::BoxDev *>(work + o_boxes);
  auto *d_tfirst = reinterpret_cast<long long *>(work + o_tfirst);
  auto *d_max = reinterpret_cast<unsigned long long *>(work + o_max);
  auto *d_dep = reinterpret_cast<unsigned long long *>(work + o_dep);
  auto *scratch = static_cast<unsigned long long *>(ctx->box_scratch.p);
  auto *counters = static_cast<unsigned long long *>(ctx->counters.p);
  hipStream_t st = ctx->stream;
  HIP_TRY(ctx, copy_sync(ctx, d_boxes, bd.data(), sizeof(pmc::BoxDev) * bd.size(), hipMemcpyHostToDevice),
          "upload boxes");
  auto *d_items = reinterpret_cast<WorkItem *>(work + o_items);
  if (!bitems.empty())
    HIP_TRY(ctx, copy_sync(ctx, d_items, bitems.data(), sizeof(WorkItem) * bitems.size(),
                           hipMemcpyHostToDevice), "upload batch work items");
  auto *d_cores = reinterpret_cast<pmc::CoreDev *>(work + o_cores);
  auto *d_slices = reinterpret_cast<pmc::SliceCore *>(work + o_cores);
  if (!cores.empty())
    HIP_TRY(ctx, copy_sync(ctx, d_cores, cores.data(), sizeof(pmc::CoreDev) * cores.size(),
                           hipMemcpyHostToDevice), "upload core windows");
  if (!slices.empty())
    HIP_TRY(ctx, copy_sync(ctx, d_slices, slices.data(), sizeof(pmc::SliceCore) * slices.size(),
                           hipMemcpyHostToDevice), "upload slice cores");
  HIP_TRY(ctx, pmc::launch_fill_u64(counters, PMC_COUNTERS, 0ull, st), "counter reset");
  unsigned __int128 deposited = 0;
  uint64_t nnz = 0;
  std::vector<long long> tfirst((size_t)max_spots + 1);
  unsigned long long *no_tally[1] = {nullptr};
  for (size_t b = 0; b + 1 < cuts.size(); ++b) {
    const int64_t s0 = cuts[b], s1 = cuts[b + 1];
    const long long base = offset[s0], entries = offset[s1] - base;
    const long long n_tiles = entries / pmc::kTile;
    // the batch's box tallies start at zero: only entries beyond the part
    // known to be zero are filled; until this batch has cleared the tiles it
    // writes (the last pass) nothing is known to be zero
    if (entries > ctx->box_zero)
      HIP_TRY(ctx, pmc::launch_fill_u64(scratch + ctx->box_zero, entries - ctx->box_zero, 0ull, st),
              "zero box tallies");
    const long long zero_after = std::max(ctx->box_zero, entries);
    ctx->box_zero = 0;
    HIP_TRY(ctx, pmc::launch_fill_u64(d_max, s1 - s0, 0ull, st), "zero maxima");
    HIP_TRY(ctx, pmc::launch_fill_u64(d_dep, 2, 0ull, st), "zero sums");
    if (batch_first[b + 1] > batch_first[b]) {
      pmc_request br = rq;
      unsigned long long *cursor = nullptr;
      hipEvent_t *cursor_done = nullptr;
      rc = take_cursor(ctx, st, &cursor, &cursor_done);
      if (rc) return rc;
      const BoxArgs ba = {d_boxes, scratch, base, d_items + batch_first[b],
                          (int32_t)(batch_first[b + 1] - batch_first[b]),
                          core_cap > 0 && !slanted ? d_cores : nullptr, core_cap,
                          core_cap > 0 && slanted ? d_slices : nullptr};
      rc = enqueue_prepared<R>(ctx, *P, &br, st, no_tally, counters, static_cast<unsigned char *>(P->buf.p),
                               cursor, true, &ba);
      if (rc) return rc;
      HIP_TRY(ctx, hipEventRecord(*cursor_done, st), "hipEventRecord");
    }
    for (int64_t s = s0; s <= s1; ++s) tfirst[s - s0] = (offset[s] - base) / pmc::kTile;
    HIP_TRY(ctx, hipMemcpyAsync(d_tfirst, tfirst.data(), sizeof(long long) * (size_t)(s1 - s0 + 1),
                                hipMemcpyHostToDevice, st), "upload tile offsets");
    pmc::InfluenceLaunch L;
    L.box_tally = reinterpret_cast<const long long *>(scratch);
    L.boxes = d_boxes + s0;
    L.tile_first = d_tfirst;
    L.n_spots = (int32_t)(s1 - s0);
    L.n_tiles = n_tiles;
    L.box_bias = base;
    L.hu = ph.d_hu;
    L.mask = ph.d_mask;
    L.lut64 = ph.d_lut64;
    L.nx = ph.nx;
    L.ny = ph.ny;
    L.vol_cm3 = (0.1 * ph.sp_mm[0]) * (0.1 * ph.sp_mm[1]) * (0.1 * ph.sp_mm[2]);
    L.rel_threshold = thr;
    L.spot_max = d_max;
    L.dep_sum = d_dep;
    L.tile_count = reinterpret_cast<uint32_t *>(work + o_count);
    L.tile_keep = L.tile_count + n_tiles;
    HIP_TRY(ctx, pmc::launch_fill_u64(reinterpret_cast<unsigned long long *>(L.tile_count), n_tiles, 0ull, st),
            "zero tile counts");  // 2 x n_tiles 32-bit words
    L.tile_off = reinterpret_cast<unsigned long long *>(work + o_toff);
    L.chunk_off = reinterpret_cast<unsigned long long *>(work + o_coff);
    L.nnz_base = (long long)nnz;
    L.row_ptr = static_cast<int64_t *>(ctx->inf_rows.p) + s0;
    L.voxel = nullptr;
    L.value = nullptr;
    HIP_TRY(ctx, pmc::launch_influence_reduce(L, st), "influence reduction");
    const long long n_chunks = (n_tiles + 1023) / 1024;
    uint64_t hostv[3] = {0, 0, 0};
    HIP_TRY(ctx, hipMemcpyAsync(hostv, L.chunk_off + n_chunks, sizeof(uint64_t), hipMemcpyDeviceToHost, st),
            "read batch size");
    HIP_TRY(ctx, hipMemcpyAsync(hostv + 1, d_dep, 2 * sizeof(uint64_t), hipMemcpyDeviceToHost, st),
            "read batch sum");
    HIP_TRY(ctx, hipStreamSynchronize(st), "influence batch");
    deposited += ((unsigned __int128)hostv[2] << 64) | hostv[1];
    rc = grow_csr(ctx, (size_t)(nnz + hostv[0]), st);
    if (rc) return rc;
    L.voxel = static_cast<int32_t *>(ctx->inf_voxel.p);
    L.value = static_cast<float *>(ctx->inf_value.p);
    HIP_TRY(ctx, pmc::launch_influence_write(L, st), "influence write");
    ctx->box_zero = zero_after;  // the write pass ends by clearing every tile with energy
    nnz += hostv[0];
    ctx->inf_nnz = nnz;
  }
  const int64_t last = (int64_t)nnz;
  HIP_TRY(ctx, hipMemcpyAsync(static_cast<int64_t *>(ctx->inf_rows.p) + n_spots, &last, sizeof last,
                              hipMemcpyHostToDevice, st), "row end");
  uint64_t c[PMC_COUNTERS];
  HIP_TRY(ctx, hipMemcpyAsync(c, counters, sizeof c, hipMemcpyDeviceToHost, st), "read counters");
  HIP_TRY(ctx, hipStreamSynchronize(st), "influence");
  rc = note_use(ctx, P->uses, st);
  if (rc) return rc;
  ctx->inf_n_rows = n_spots;
  ctx->inf_nnz = nnz;
  *nnz_out = nnz;
  if (bal_out) fill_balance(P->incident, c, deposited, bal_out);
  if (outside_out) {
    outside_out[0] = c[13];
    outside_out[1] = c[14];
  }
  return PMC_OK;
}

}  // namespace

extern "C" {

int pmc_influence_boxes(pmc_context *ctx, int32_t plan, int32_t phase, pmc_box *out, int64_t n_spots) {
  if (!ctx) return fail(nullptr, PMC_E_INVAL, "context is NULL");
  ctx->err.clear();
  auto pit = ctx->plans.find(plan);
  if (pit == ctx->plans.end()) return fail(ctx, PMC_E_STATE, "plan %d is not loaded", plan);
  auto hit = ctx->phases.find(phase);
  if (hit == ctx->phases.end()) return fail(ctx, PMC_E_NOPHASE, "phase %d is not loaded", phase);
  if (!out || n_spots != (int64_t)pit->second.spots.size())
    return fail(ctx, PMC_E_INVAL, "need an output array of the plan's %zu spots", pit->second.spots.size());
  const PlanRec &P = pit->second;
  parallel_for(n_spots, [&](int64_t s) {
    out[s] = P.spots[s].phase == phase ? spot_box(ctx, hit->second, P.fields[P.spots[s].field], P.spots[s])
                                       : pmc_box{{0, 0, 0}, {0, 0, 0}};
  });
  return PMC_OK;
}

int pmc_influence(pmc_context *ctx, const pmc_request *req, const pmc_box *boxes, double rel_threshold,
                  uint64_t max_scratch_bytes, uint64_t *nnz, pmc_balance *balance, uint64_t outside[2]) {
  if (!ctx) return fail(nullptr, PMC_E_INVAL, "context is NULL");
  ctx->err.clear();
  int rc = validate_request(ctx, req);
  if (rc) return rc;
  if (!nnz) return fail(ctx, PMC_E_INVAL, "nnz is NULL");
  if (req->n_phases != 1) return fail(ctx, PMC_E_INVAL, "an influence request has exactly one phase");
  if (req->item_begin || req->item_end) return fail(ctx, PMC_E_INVAL, "an influence request is not sliced");
  if (!(rel_threshold >= 0.0 && rel_threshold <= 1.0))
    return fail(ctx, PMC_E_INVAL, "rel_threshold must be in [0, 1]");
  if (!ctx->has_device) return fail(ctx, PMC_E_DEVICE, "validation-only context has no device");
  HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  rc = ctx->precision == PMC_FP64
           ? influence<double>(ctx, req, boxes, rel_threshold, max_scratch_bytes, nnz, balance, outside)
           : influence<float>(ctx, req, boxes, rel_threshold, max_scratch_bytes, nnz, balance, outside);
  if (rc) {
    (void)hipStreamSynchronize(ctx->stream);
    ctx->inf_n_rows = -1;
  }
  return rc;
}

int pmc_influence_read(pmc_context *ctx, int64_t *row_ptr, int32_t *voxel, float *value) {
  if (!ctx) return fail(nullptr, PMC_E_INVAL, "context is NULL");
  ctx->err.clear();
  if (ctx->inf_n_rows < 0) return fail(ctx, PMC_E_STATE, "no influence matrix has been computed");
  if (row_ptr)
    HIP_TRY(ctx, copy_sync(ctx, row_ptr, ctx->inf_rows.p, sizeof(int64_t) * (size_t)(ctx->inf_n_rows + 1),
                           hipMemcpyDeviceToHost), "copy rows");
  if (voxel && ctx->inf_nnz)
    HIP_TRY(ctx, copy_sync(ctx, voxel, ctx->inf_voxel.p, sizeof(int32_t) * ctx->inf_nnz, hipMemcpyDeviceToHost),
            "copy voxels");
  if (value && ctx->inf_nnz)
    HIP_TRY(ctx, copy_sync(ctx, value, ctx->inf_value.p, sizeof(float) * ctx->inf_nnz, hipMemcpyDeviceToHost),
            "copy values");
  return PMC_OK;
}

int pmc_influence_device(pmc_context *ctx, const int64_t **row_ptr, const int32_t **voxel, const float **value) {
  if (!ctx) return fail(nullptr, PMC_E_INVAL, "context is NULL");
  ctx->err.clear();
  if (ctx->inf_n_rows < 0) return fail(ctx, PMC_E_STATE, "no influence matrix has been computed");
  if (row_ptr) *row_ptr = static_cast<const int64_t *>(ctx->inf_rows.p);
  if (voxel) *voxel = static_cast<const int32_t *>(ctx->inf_voxel.p);
  if (value) *value = static_cast<const float *>(ctx->inf_value.p);
  return PMC_OK;
}

int pmc_influence_free(pmc_context *ctx) {
  if (!ctx) return fail(nullptr, PMC_E_INVAL, "context is NULL");
  ctx->err.clear();
  if (ctx->has_device) {
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
  }
  free_influence(ctx);
  return PMC_OK;
}

}  // extern "C"

// ===========================================================================
// deformable dose accumulation (Sec. 2.D.2, energy/mass transfer; App. B)
// ===========================================================================

int pmc_load_dvf(pmc_context *ctx, int32_t dvf, const pmc_dvf *d) {
  if (!ctx) return fail(nullptr, PMC_E_INVAL, "context is NULL");
  ctx->err.clear();
  if (dvf < 0 || dvf > kMaxPhaseId) return fail(ctx, PMC_E_INVAL, "dvf id must be 0..%d", kMaxPhaseId);
  if (!d || !d->delta_mm) return fail(ctx, PMC_E_INVAL, "NULL DVF");
  for (int k = 0; k < 3; ++k) {
    if (d->n[k] < 2) return fail(ctx, PMC_E_INVAL, "a DVF grid needs >= 2 points along every axis");
    if (!(std::isfinite(d->spacing_mm[k]) && d->spacing_mm[k] > 0.0))
      return fail(ctx, PMC_E_INVAL, "DVF spacing must be finite and > 0");
  }
  if (!finite3(d->start_mm) || !finite3(d->row) || !finite3(d->col))
    return fail(ctx, PMC_E_INVAL, "DVF start and directions must be finite");
  const double nr = norm3(d->row), nc = norm3(d->col);
  const double dot = d->row[0] * d->col[0] + d->row[1] * d->col[1] + d->row[2] * d->col[2];
  if (std::fabs(nr - 1.0) > 1e-6 || std::fabs(nc - 1.0) > 1e-6 || std::fabs(dot) > 1e-6)
    return fail(ctx, PMC_E_INVAL, "DVF row and column directions must be orthonormal");
  // rigid 4x4 matrices of Eq. (7): rotation part orthonormal, last row 0 0 0 1
  auto check_rigid = [&](const double *m, const char *name) -> int {
    for (int i = 0; i < 16; ++i)
      if (!std::isfinite(m[i])) return fail(ctx, PMC_E_INVAL, "%s has a non-finite entry", name);
    if (m[12] != 0.0 || m[13] != 0.0 || m[14] != 0.0 || m[15] != 1.0)
      return fail(ctx, PMC_E_INVAL, "%s must have the last row 0 0 0 1", name);
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        const double dot = m[4 * r] * m[4 * c] + m[4 * r + 1] * m[4 * c + 1] + m[4 * r + 2] * m[4 * c + 2];
        if (std::fabs(dot - (r == c ? 1.0 : 0.0)) > 1e-6)
          return fail(ctx, PMC_E_INVAL, "%s must be rigid (orthonormal rotation part)", name);
      }
    return PMC_OK;
  };
  if (d->pre) {
    int rc = check_rigid(d->pre, "M_pre");
    if (rc) return rc;
  }
  if (d->post) {
    int rc = check_rigid(d->post, "M_post");
    if (rc) return rc;
  }
  const long long pts = (long long)d->n[0] * d->n[1] * d->n[2];
  if (pts > (1LL << 31)) return fail(ctx, PMC_E_INVAL, "DVF grid has more than 2^31 points");
  for (long long i = 0; i < 3 * pts; ++i)
    if (!std::isfinite(d->delta_mm[i])) return fail(ctx, PMC_E_INVAL, "DVF translation %lld is not finite", i / 3);
  DvfRec rec;
  pmc::DvfDev &g = rec.dev;
  for (int k = 0; k < 3; ++k) {
    g.n[k] = d->n[k];
    g.start[k] = d->start_mm[k];
    g.sp[k] = d->spacing_mm[k];
    g.u[k] = d->row[k];
    g.v[k] = d->col[k];
  }
  // depth direction W = U x V (Eq. (8))
  g.w[0] = g.u[1] * g.v[2] - g.u[2] * g.v[1];
  g.w[1] = g.u[2] * g.v[0] - g.u[0] * g.v[2];
  g.w[2] = g.u[0] * g.v[1] - g.u[1] * g.v[0];
  g.has_pre = d->pre != nullptr;
  g.has_post = d->post != nullptr;
  for (int i = 0; i < 12; ++i) {
    g.pre[i] = d->pre ? d->pre[i] : 0.0;
    g.post[i] = d->post ? d->post[i] : 0.0;
  }
  rec.bytes = sizeof(double) * 3 * (size_t)pts;
  if (ctx->has_device) {
    HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    int rc = pool_get(ctx, rec.bytes, &rec.d_delta, &rec.cap, "DVF translations");
    if (rc) return rc;
    hipError_t e = copy_sync(ctx, rec.d_delta, d->delta_mm, rec.bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      pool_put(ctx, rec.d_delta, rec.cap);
      return hip_fail(ctx, e, "upload DVF");
    }
    g.delta = static_cast<const double *>(rec.d_delta);
  }
  auto it = ctx->dvfs.find(dvf);
  if (it != ctx->dvfs.end()) {
    wait_use(it->second.uses);
    drop_use(it->second.uses);
    pool_put(ctx, it->second.d_delta, it->second.cap);
    ctx->dvfs.erase(it);
  }
  ctx->dvfs[dvf] = std::move(rec);
  return PMC_OK;
}

int pmc_unload_dvf(pmc_context *ctx, int32_t dvf) {
  if (!ctx) return fail(nullptr, PMC_E_INVAL, "context is NULL");
  ctx->err.clear();
  auto it = ctx->dvfs.find(dvf);
  if (it == ctx->dvfs.end()) return fail(ctx, PMC_E_STATE, "dvf %d is not loaded", dvf);
  wait_use(it->second.uses);
  drop_use(it->second.uses);
  pool_put(ctx, it->second.d_delta, it->second.cap);
  ctx->dvfs.erase(it);
  return PMC_OK;
}

int pmc_dvf_points(pmc_context *ctx, int32_t dvf, double *x0_out, double *rf_out) {
  if (!ctx) return fail(nullptr, PMC_E_INVAL, "context is NULL");
  ctx->err.clear();
  auto it = ctx->dvfs.find(dvf);
  if (it == ctx->dvfs.end()) return fail(ctx, PMC_E_STATE, "dvf %d is not loaded", dvf);
  if (!ctx->has_device) return fail(ctx, PMC_E_DEVICE, "validation-only context has no device");
  if (!x0_out && !rf_out) return PMC_OK;
  HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  const pmc::DvfDev &g = it->second.dev;
  const size_t bytes = sizeof(double) * 3 * (size_t)g.n[0] * g.n[1] * g.n[2];
  void *d_x0 = nullptr, *d_rf = nullptr;
  size_t c_x0 = 0, c_rf = 0;
  auto cleanup = [&](int code) {
    (void)hipStreamSynchronize(ctx->stream);
    if (d_x0) pool_put(ctx, d_x0, c_x0);
    if (d_rf) pool_put(ctx, d_rf, c_rf);
    return code;
  };
  int rc = x0_out ? pool_get(ctx, bytes, &d_x0, &c_x0, "DVF points") : PMC_OK;
  if (!rc && rf_out) rc = pool_get(ctx, bytes, &d_rf, &c_rf, "DVF points");
  if (rc) return cleanup(rc);
  hipError_t e = pmc::launch_dvf_points(g, static_cast<double *>(d_x0), static_cast<double *>(d_rf), ctx->stream);
  if (e != hipSuccess) return cleanup(hip_fail(ctx, e, "dvf_points launch"));
  if (x0_out) e = copy_sync(ctx, x0_out, d_x0, bytes, hipMemcpyDeviceToHost);
  if (e == hipSuccess && rf_out) e = copy_sync(ctx, rf_out, d_rf, bytes, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return cleanup(hip_fail(ctx, e, "download DVF points"));
  return cleanup(PMC_OK);
}

namespace {

int validate_accumulate(pmc_context *ctx, int32_t ref_phase, int32_t n_src, const int32_t *src_phases,
                        const int32_t *src_dvfs, int32_t n_sub, uint64_t n_histories) {
  if (ctx->phases.find(ref_phase) == ctx->phases.end())
    return fail(ctx, PMC_E_NOPHASE, "reference phase %d is not loaded", ref_phase);
  if (n_src < 0 || n_src > PMC_MAX_PHASES) return fail(ctx, PMC_E_INVAL, "n_src must be 0..%d", PMC_MAX_PHASES);
  if (n_src > 0 && (!src_phases || !src_dvfs)) return fail(ctx, PMC_E_INVAL, "NULL source list");
  for (int32_t s = 0; s < n_src; ++s) {
    if (ctx->phases.find(src_phases[s]) == ctx->phases.end())
      return fail(ctx, PMC_E_NOPHASE, "source phase %d is not loaded", src_phases[s]);
    if (ctx->dvfs.find(src_dvfs[s]) == ctx->dvfs.end())
      return fail(ctx, PMC_E_STATE, "dvf %d is not loaded", src_dvfs[s]);
  }
  if (n_sub < 1 || n_sub > 16) return fail(ctx, PMC_E_INVAL, "n_sub must be 1..16");
  if (n_histories == 0) return fail(ctx, PMC_E_INVAL, "n_histories must be >= 1");
  const PhaseRec &ref = ctx->phases[ref_phase];
  if (ref.nx >= (1 << 20) - 1 || ref.ny >= (1 << 20) - 1 || ref.nz >= (1 << 20) - 1)
    return fail(ctx, PMC_E_INVAL, "reference grid needs fewer than 2^20 - 1 voxels per axis");
  return PMC_OK;
}

}  // namespace

namespace {

enum AccMethod { kEmtm = 0, kDim = 1 };

bool aligned_dvf(const pmc::DvfDev &g) {
  return g.u[0] == 1.0 && g.u[1] == 0.0 && g.u[2] == 0.0 && g.v[0] == 0.0 && g.v[1] == 1.0 && g.v[2] == 0.0 &&
         !g.has_pre && !g.has_post;
}

pmc::DvfBox box_of(const pmc::DvfDev &g) {
  pmc::DvfBox b = {};
  for (int k = 0; k < 3; ++k) {
    b.n[k] = g.n[k];
    b.start[k] = g.start[k];
    b.sp[k] = g.sp[k];
    b.u[k] = g.u[k];
    b.v[k] = g.v[k];
    b.w[k] = g.w[k];
  }
  return b;
}

int accumulate_device(pmc_context *ctx, AccMethod method, int32_t ref_phase, const int64_t *ref_tally,
                      int32_t n_src, const int32_t *src_phases, const int32_t *src_dvfs,
                      const int64_t *const *src_tallies, int32_t n_sub, uint64_t n_histories, void *stream,
                      double *dev_dose, uint8_t *dev_mask) {
  if (!ctx) return fail(nullptr, PMC_E_INVAL, "context is NULL");
  ctx->err.clear();
  int rc = validate_accumulate(ctx, ref_phase, n_src, src_phases, src_dvfs, n_sub, n_histories);
  if (rc) return rc;
  if (!ref_tally || !dev_dose) return fail(ctx, PMC_E_INVAL, "need the reference tally and a dose buffer");
  if (n_src > 0 && !src_tallies) return fail(ctx, PMC_E_INVAL, "NULL source tallies");
  for (int32_t s = 0; s < n_src; ++s)
    if (!src_tallies[s]) return fail(ctx, PMC_E_INVAL, "source tally %d is NULL", s);
  if (!ctx->has_device) return fail(ctx, PMC_E_DEVICE, "validation-only context has no device");
  HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  hipStream_t st = static_cast<hipStream_t>(stream);
  PhaseRec &ref = ctx->phases[ref_phase];
  const long long nvox = ref.nvox();
  const double vol_ref = (0.1 * ref.sp_mm[0]) * (0.1 * ref.sp_mm[1]) * (0.1 * ref.sp_mm[2]);
  const double nh = (double)n_histories;
  // D^R: the reference phase's own dose (Eq. (2), first term)
  HIP_TRY(ctx, pmc::launch_convert((const long long *)ref_tally, ref.d_hu, ref.d_mask, ref.d_lut64, nvox,
                                   vol_ref, nh, dev_dose, nullptr, st),
          "reference dose");
  if (n_src > 0 && method == kDim) {
    // scratch: one source dose at a time; wait (on this stream) for the calls
    // that used the scratch before
    size_t need = 0;
    for (int32_t s = 0; s < n_src; ++s)
      need = std::max(need, sizeof(double) * (size_t)ctx->phases[src_phases[s]].nvox());
    rc = ensure(ctx, ctx->acc, need, "accumulators");
    if (rc) return rc;
    for (auto &p : ctx->acc_uses.ev) HIP_TRY(ctx, hipStreamWaitEvent(st, p.second, 0), "wait accumulators");
    auto *sdose = static_cast<double *>(ctx->acc.p);
    for (int32_t s = 0; s < n_src; ++s) {
      const PhaseRec &src = ctx->phases[src_phases[s]];
      const DvfRec &dv = ctx->dvfs[src_dvfs[s]];
      const double vol_src = (0.1 * src.sp_mm[0]) * (0.1 * src.sp_mm[1]) * (0.1 * src.sp_mm[2]);
      HIP_TRY(ctx, pmc::launch_convert((const long long *)src_tallies[s], src.d_hu, src.d_mask, src.d_lut64,
                                       src.nvox(), vol_src, nh, sdose, nullptr, st),
              "source dose");
      pmc::DimPull a = {};
      a.nx = ref.nx;
      a.ny = ref.ny;
      a.nz = ref.nz;
      a.dvf = dv.dev;
      a.snx = src.nx;
      a.sny = src.ny;
      a.snz = src.nz;
      for (int k = 0; k < 3; ++k) {
        a.org[k] = ref.org_mm[k];
        a.sp[k] = ref.sp_mm[k];
        a.sorg[k] = src.org_mm[k];
        a.ssp[k] = src.sp_mm[k];
      }
      a.sdose = sdose;
      a.n_sub = n_sub;
      a.aligned = aligned_dvf(dv.dev);
      a.dose = dev_dose;
      HIP_TRY(ctx, pmc::launch_dim_pull(a, st), "dim_pull launch");
    }
  } else if (n_src > 0) {
    // accumulators: wait (on this stream) for the calls that used them before
    rc = ensure(ctx, ctx->acc, 3 * sizeof(unsigned long long) * (size_t)nvox, "accumulators");
    if (rc) return rc;
    for (auto &p : ctx->acc_uses.ev) HIP_TRY(ctx, hipStreamWaitEvent(st, p.second, 0), "wait accumulators");
    auto *e_hi = static_cast<unsigned long long *>(ctx->acc.p);
    auto *e_lo = e_hi + nvox, *mass = e_lo + nvox;
    for (int32_t s = 0; s < n_src; ++s) {
      const PhaseRec &src = ctx->phases[src_phases[s]];
      const DvfRec &dv = ctx->dvfs[src_dvfs[s]];
      HIP_TRY(ctx, pmc::launch_fill_u64(e_hi, 3 * nvox, 0ull, st), "zero accumulators");
      pmc::EmtmPush a = {};
      a.hu = src.d_hu;
      a.mask = src.d_mask;
      a.lut64 = static_cast<const double *>(src.d_lut64);
      a.tally = (const long long *)src_tallies[s];
      a.nx = src.nx;
      a.ny = src.ny;
      a.nz = src.nz;
      a.dvf = dv.dev;
      a.rnx = ref.nx;
      a.rny = ref.ny;
      a.rnz = ref.nz;
      for (int k = 0; k < 3; ++k) {
        a.org[k] = src.org_mm[k];
        a.sp[k] = src.sp_mm[k];
        a.rorg[k] = ref.org_mm[k];
        a.rsp[k] = ref.sp_mm[k];
        a.rinv[k] = 1.0 / ref.sp_mm[k];
      }
      a.n_sub = n_sub;
      a.aligned = aligned_dvf(dv.dev);
      a.e_hi = e_hi;
      a.e_lo = e_lo;
      a.mass = mass;
      HIP_TRY(ctx, pmc::launch_emtm_push(a, st), "emtm_push launch");
      pmc::EmtmRatio r = {};
      r.e_hi = e_hi;
      r.e_lo = e_lo;
      r.mass = mass;
      r.dose = dev_dose;
      r.nvox = nvox;
      r.vol_cm3 = (0.1 * src.sp_mm[0]) * (0.1 * src.sp_mm[1]) * (0.1 * src.sp_mm[2]);
      r.n_hist = nh;
      HIP_TRY(ctx, pmc::launch_emtm_ratio(r, st), "emtm_ratio launch");
    }
  }
  // report mask: the reference voxel centres inside every DVF's grid box
  for (int32_t s0 = 0; s0 < n_src || (s0 == 0 && dev_mask); s0 += pmc::kMaskDvfs) {
    pmc::EmtmMask m = {};
    m.n_dvf = std::min<int32_t>(pmc::kMaskDvfs, n_src - s0);
    for (int32_t k = 0; k < m.n_dvf; ++k) m.dvfs[k] = box_of(ctx->dvfs[src_dvfs[s0 + k]].dev);
    m.first = s0 == 0;
    m.nx = ref.nx;
    m.ny = ref.ny;
    m.nz = ref.nz;
    for (int k = 0; k < 3; ++k) {
      m.org[k] = ref.org_mm[k];
      m.sp[k] = ref.sp_mm[k];
    }
    m.dose = dev_dose;
    m.mask_out = dev_mask;
    HIP_TRY(ctx, pmc::launch_emtm_mask(m, st), "emtm_mask launch");
    if (n_src == 0) break;
  }
  // the inputs read by this call stay alive until it has run
  rc = note_use(ctx, ref.uses, st);
  for (int32_t s = 0; s < n_src && !rc; ++s) {
    rc = note_use(ctx, ctx->phases[src_phases[s]].uses, st);
    if (!rc) rc = note_use(ctx, ctx->dvfs[src_dvfs[s]].uses, st);
  }
  if (!rc && n_src > 0) rc = note_use(ctx, ctx->acc_uses, st);
  if (rc) return rc;
  return note_pending(ctx, st);
}

int accumulate_host(pmc_context *ctx, AccMethod method, int32_t ref_phase, const int64_t *ref_tally,
                    int32_t n_src, const int32_t *src_phases, const int32_t *src_dvfs,
                    const int64_t *const *src_tallies, int32_t n_sub, uint64_t n_histories, double *dose_out,
                    uint8_t *mask_out) {
  if (!ctx) return fail(nullptr, PMC_E_INVAL, "context is NULL");
  ctx->err.clear();
  int rc = validate_accumulate(ctx, ref_phase, n_src, src_phases, src_dvfs, n_sub, n_histories);
  if (rc) return rc;
  if (!ref_tally || !dose_out) return fail(ctx, PMC_E_INVAL, "need the reference tally and a dose buffer");
  if (n_src > 0 && !src_tallies) return fail(ctx, PMC_E_INVAL, "NULL source tallies");
  for (int32_t s = 0; s < n_src; ++s)
    if (!src_tallies[s]) return fail(ctx, PMC_E_INVAL, "source tally %d is NULL", s);
  if (!ctx->has_device) return fail(ctx, PMC_E_DEVICE, "validation-only context has no device");
  HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  // device copies of the tallies (source grids may differ from the reference)
  struct Block { void *p = nullptr; size_t cap = 0; };
  std::vector<Block> blocks;
  auto cleanup = [&](int code) {
    (void)hipStreamSynchronize(ctx->stream);
    for (auto &b : blocks) pool_put(ctx, b.p, b.cap);
    return code;
  };
  auto upload = [&](const void *src, size_t bytes, void **dst) -> int {
    Block b;
    int r = pool_get(ctx, std::max<size_t>(bytes, 256), &b.p, &b.cap, "accumulation inputs");
    if (r) return r;
    blocks.push_back(b);
    *dst = b.p;
    if (src) {
      hipError_t e = copy_sync(ctx, b.p, src, bytes, hipMemcpyHostToDevice);
      if (e != hipSuccess) return hip_fail(ctx, e, "upload tally");
    }
    return PMC_OK;
  };
  const PhaseRec &ref = ctx->phases[ref_phase];
  const long long nvox = ref.nvox();
  void *d_ref = nullptr, *d_dose = nullptr, *d_mask = nullptr;
  rc = upload(ref_tally, sizeof(int64_t) * (size_t)nvox, &d_ref);
  std::vector<const int64_t *> d_src((size_t)n_src, nullptr);
  for (int32_t s = 0; s < n_src && !rc; ++s) {
    void *p = nullptr;
    rc = upload(src_tallies[s], sizeof(int64_t) * (size_t)ctx->phases[src_phases[s]].nvox(), &p);
    d_src[s] = static_cast<const int64_t *>(p);
  }
  if (!rc) rc = upload(nullptr, sizeof(double) * (size_t)nvox, &d_dose);
  if (!rc && mask_out) rc = upload(nullptr, (size_t)nvox, &d_mask);
  if (rc) return cleanup(rc);
  rc = accumulate_device(ctx, method, ref_phase, static_cast<const int64_t *>(d_ref), n_src, src_phases, src_dvfs,
                         d_src.data(), n_sub, n_histories, ctx->stream, static_cast<double *>(d_dose),
                         static_cast<uint8_t *>(d_mask));
  if (rc) return cleanup(rc);
  hipError_t e = copy_sync(ctx, dose_out, d_dose, sizeof(double) * (size_t)nvox, hipMemcpyDeviceToHost);
  if (e == hipSuccess && mask_out) e = copy_sync(ctx, mask_out, d_mask, (size_t)nvox, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return cleanup(hip_fail(ctx, e, "download accumulated dose"));
  return cleanup(PMC_OK);
}

}  // namespace

int pmc_accumulate_device(pmc_context *ctx, int32_t ref_phase, const int64_t *ref_tally, int32_t n_src,
                          const int32_t *src_phases, const int32_t *src_dvfs, const int64_t *const *src_tallies,
                          int32_t n_sub, uint64_t n_histories, void *stream, double *dev_dose,
                          uint8_t *dev_mask) {
  return accumulate_device(ctx, kEmtm, ref_phase, ref_tally, n_src, src_phases, src_dvfs, src_tallies, n_sub,
                           n_histories, stream, dev_dose, dev_mask);
}

int pmc_accumulate_dim_device(pmc_context *ctx, int32_t ref_phase, const int64_t *ref_tally, int32_t n_src,
                              const int32_t *src_phases, const int32_t *src_dvfs,
                              const int64_t *const *src_tallies, int32_t n_sub, uint64_t n_histories,
                              void *stream, double *dev_dose, uint8_t *dev_mask) {
  return accumulate_device(ctx, kDim, ref_phase, ref_tally, n_src, src_phases, src_dvfs, src_tallies, n_sub,
                           n_histories, stream, dev_dose, dev_mask);
}

int pmc_accumulate(pmc_context *ctx, int32_t ref_phase, const int64_t *ref_tally, int32_t n_src,
                   const int32_t *src_phases, const int32_t *src_dvfs, const int64_t *const *src_tallies,
                   int32_t n_sub, uint64_t n_histories, double *dose_out, uint8_t *mask_out) {
  return accumulate_host(ctx, kEmtm, ref_phase, ref_tally, n_src, src_phases, src_dvfs, src_tallies, n_sub,
                         n_histories, dose_out, mask_out);
}

int pmc_accumulate_dim(pmc_context *ctx, int32_t ref_phase, const int64_t *ref_tally, int32_t n_src,
                       const int32_t *src_phases, const int32_t *src_dvfs, const int64_t *const *src_tallies,
                       int32_t n_sub, uint64_t n_histories, double *dose_out, uint8_t *mask_out) {
  return accumulate_host(ctx, kDim, ref_phase, ref_tally, n_src, src_phases, src_dvfs, src_tallies, n_sub,
                         n_histories, dose_out, mask_out);
}

// ---------------------------------------------------------------------------
// beam-delivery simulation (Sec. 2.B, App. A)
// ---------------------------------------------------------------------------

int pmc_delivery_simulate(pmc_context *ctx, const pmc_delivery *d, const pmc_spot *spots, int64_t n_spots,
                          int32_t n_fields, double *mu_out, double *time_out, int32_t *fills_out) {
  if (!ctx) return fail(nullptr, PMC_E_INVAL, "context is NULL");
  ctx->err.clear();
  if (!d || (!spots && n_spots > 0)) return fail(ctx, PMC_E_INVAL, "NULL delivery options or spots");
  if (d->n_phases < 1 || d->n_phases > 64) return fail(ctx, PMC_E_INVAL, "n_phases must be 1..64");
  if (d->start_phase < -1 || d->start_phase >= d->n_phases)
    return fail(ctx, PMC_E_INVAL, "start_phase must be -1 or 0..n_phases-1");
  const bool random_period = d->period_min_s > 0 && d->period_min_s <= d->period_max_s;
  if (d->period_min_s < 0 || d->period_max_s < 0 || d->period_max_s > 3600)
    return fail(ctx, PMC_E_INVAL, "period_min_s/period_max_s must be 0..3600");
  if (!random_period && !(std::isfinite(d->period_s) && d->period_s > 0.0))
    return fail(ctx, PMC_E_INVAL, "period_s must be finite and > 0");
  if (!(std::isfinite(d->period_sd_s) && d->period_sd_s >= 0.0))
    return fail(ctx, PMC_E_INVAL, "period_sd_s must be finite and >= 0");
  if (d->gate_lo != -1 && !(d->gate_lo >= 0 && d->gate_lo <= d->gate_hi && d->gate_hi < d->n_phases))
    return fail(ctx, PMC_E_INVAL, "gate must be -1 or 0 <= gate_lo <= gate_hi < n_phases");
  if (!(std::isfinite(d->max_mu) && d->max_mu >= 0.0)) return fail(ctx, PMC_E_INVAL, "max_mu must be >= 0");
  if (d->n_trials < 1 || n_fields < 1 || n_spots < 0 || n_spots >= (1LL << 31))
    return fail(ctx, PMC_E_INVAL, "need n_trials >= 1, n_fields >= 1 and 0..2^31-1 spots");
  if ((long long)d->n_trials * n_fields >= (1LL << 31))
    return fail(ctx, PMC_E_INVAL, "n_trials x n_fields must be below 2^31");
  const pmc_param *par = &d->sync.layer_switch_s;
  for (int i = 0; i < pmc::kSyncParams; ++i)
    if (!(std::isfinite(par[i].central) && std::isfinite(par[i].sd) && par[i].sd >= 0.0))
      return fail(ctx, PMC_E_INVAL, "synchrotron parameter %d must be finite with sd >= 0", i);
  const double out_bytes = (double)d->n_trials * (double)n_spots * (double)d->n_phases * 8.0;
  if (out_bytes > 64e9) return fail(ctx, PMC_E_INVAL, "trials x spots x phases too large");
  // spots grouped by field, plan order kept within a field; spill rates
  // positive for any draw within +-6.8 sigma (the Box-Muller deviate of two
  // 32-bit uniforms never leaves +-6.77)
  std::vector<int32_t> fstart((size_t)n_fields + 1, 0);
  for (int64_t i = 0; i < n_spots; ++i) {
    const pmc_spot &sp = spots[i];
    if (sp.field < 0 || sp.field >= n_fields) return fail(ctx, PMC_E_INVAL, "spot %lld: bad field", (long long)i);
    if (!(std::isfinite(sp.energy_MeV) && sp.energy_MeV >= 1.0 && sp.energy_MeV <= 300.0) ||
        !std::isfinite(sp.x_mm) || !std::isfinite(sp.y_mm) || !(std::isfinite(sp.weight) && sp.weight > 0.0))
      return fail(ctx, PMC_E_INVAL, "spot %lld: energy 1..300 MeV, finite position, MU > 0", (long long)i);
    const double de = sp.energy_MeV - 70.0;
    const double c = par[3].central - 6.8 * par[3].sd;
    const double s_lo = (par[4].central - 6.8 * par[4].sd) * de, s_hi = (par[4].central + 6.8 * par[4].sd) * de;
    if (!(c + std::min(s_lo, s_hi) > 0.0))
      return fail(ctx, PMC_E_INVAL, "spill rate can reach <= 0 at %g MeV", sp.energy_MeV);
    ++fstart[(size_t)sp.field + 1];
  }
  for (int32_t f = 0; f < n_fields; ++f) fstart[(size_t)f + 1] += fstart[(size_t)f];
  std::vector<pmc::DeliverySpot> grouped((size_t)n_spots);
  std::vector<int64_t> index((size_t)n_spots);
  {
    std::vector<int32_t> fill(fstart.begin(), fstart.end() - 1);
    for (int64_t i = 0; i < n_spots; ++i) {
      const pmc_spot &sp = spots[i];
      const int32_t at = fill[(size_t)sp.field]++;
      grouped[(size_t)at] = {sp.energy_MeV, sp.x_mm, sp.y_mm, sp.weight};
      index[(size_t)at] = i;
    }
  }
  if (!ctx->has_device) return fail(ctx, PMC_E_DEVICE, "validation-only context has no device");
  HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  const size_t n_tf = (size_t)d->n_trials * (size_t)n_fields;
  const size_t mu_bytes = (size_t)out_bytes;
  struct Block { void *p = nullptr; size_t cap = 0; };
  std::vector<Block> blocks;
  auto cleanup = [&](int code) {
    (void)hipStreamSynchronize(ctx->stream);
    for (auto &b : blocks) pool_put(ctx, b.p, b.cap);
    return code;
  };
  auto get = [&](size_t bytes, void **p) -> int {
    Block b;
    int r = pool_get(ctx, std::max<size_t>(bytes, 256), &b.p, &b.cap, "delivery simulation");
    if (r) return r;
    blocks.push_back(b);
    *p = b.p;
    return PMC_OK;
  };
  void *d_spots = nullptr, *d_fstart = nullptr, *d_index = nullptr, *d_mu = nullptr, *d_time = nullptr,
       *d_fills = nullptr, *d_status = nullptr;
  int rc = get(sizeof(pmc::DeliverySpot) * grouped.size(), &d_spots);
  if (!rc) rc = get(sizeof(int32_t) * fstart.size(), &d_fstart);
  if (!rc) rc = get(sizeof(int64_t) * index.size(), &d_index);
  if (!rc) rc = get(mu_bytes, &d_mu);
  if (!rc) rc = get(sizeof(double) * n_tf, &d_time);
  if (!rc) rc = get(sizeof(int32_t) * n_tf, &d_fills);
  if (!rc) rc = get(sizeof(int32_t), &d_status);
  if (rc) return cleanup(rc);
  hipError_t e = hipSuccess;
  if (n_spots > 0) e = copy_sync(ctx, d_spots, grouped.data(), sizeof(pmc::DeliverySpot) * grouped.size(),
                                 hipMemcpyHostToDevice);
  if (e == hipSuccess) e = copy_sync(ctx, d_fstart, fstart.data(), sizeof(int32_t) * fstart.size(),
                                     hipMemcpyHostToDevice);
  if (e == hipSuccess && n_spots > 0)
    e = copy_sync(ctx, d_index, index.data(), sizeof(int64_t) * index.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return cleanup(hip_fail(ctx, e, "upload delivery inputs"));
  if (mu_bytes >= 8) {
    e = pmc::launch_fill_u64(static_cast<unsigned long long *>(d_mu), (long long)(mu_bytes / 8), 0ull, ctx->stream);
    if (e != hipSuccess) return cleanup(hip_fail(ctx, e, "zero MU"));
  }
  {
    const int32_t zero = 0;
    e = copy_sync(ctx, d_status, &zero, sizeof(zero), hipMemcpyHostToDevice);
    if (e != hipSuccess) return cleanup(hip_fail(ctx, e, "status"));
  }
  pmc::DeliveryLaunch a = {};
  a.spots = static_cast<const pmc::DeliverySpot *>(d_spots);
  a.fstart = static_cast<const int32_t *>(d_fstart);
  a.index = static_cast<const int64_t *>(d_index);
  a.n_spots = n_spots;
  a.n_fields = n_fields;
  a.n_trials = d->n_trials;
  a.n_phases = d->n_phases;
  a.start_phase = d->start_phase;
  a.period_min = random_period ? d->period_min_s : 0;
  a.period_max = random_period ? d->period_max_s : 0;
  a.gate_lo = d->gate_lo;
  a.gate_hi = d->gate_hi;
  a.period_s = d->period_s;
  a.period_sd_s = d->period_sd_s;
  a.max_mu = d->max_mu;
  for (int i = 0; i < pmc::kSyncParams; ++i) {
    a.central[i] = par[i].central;
    a.sd[i] = par[i].sd;
  }
  a.seed = (uint32_t)(d->seed & 0xFFFFFFFFull);
  a.mu = static_cast<double *>(d_mu);
  a.time = static_cast<double *>(d_time);
  a.fills = static_cast<int32_t *>(d_fills);
  a.status = static_cast<int32_t *>(d_status);
  // longest layer, staged in LDS when it fits 64 KiB with its MU sums
  {
    int32_t longest = 0;
    for (int32_t f = 0; f < n_fields; ++f)
      for (int32_t i = fstart[(size_t)f]; i < fstart[(size_t)f + 1];) {
        int32_t j = i + 1;
        while (j < fstart[(size_t)f + 1] && grouped[(size_t)j].e == grouped[(size_t)i].e) ++j;
        longest = std::max(longest, j - i);
        i = j;
      }
    const int32_t per = (int32_t)(sizeof(pmc::DeliverySpot) + sizeof(double) * (size_t)d->n_phases);
    a.layer_cap = std::min<int32_t>(longest, 65536 / per);
  }
  e = pmc::launch_delivery(a, ctx->stream);
  if (e != hipSuccess) return cleanup(hip_fail(ctx, e, "delivery_sim launch"));
  int32_t status = 0;
  e = copy_sync(ctx, &status, d_status, sizeof(status), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return cleanup(hip_fail(ctx, e, "download delivery status"));
  // an abandoned timeline leaves the caller's buffers untouched
  if (status) return cleanup(fail(ctx, PMC_E_INVAL, "a delivery timeline exceeded 2^30 breathing phases"));
  if (mu_out && mu_bytes) e = copy_sync(ctx, mu_out, d_mu, mu_bytes, hipMemcpyDeviceToHost);
  if (e == hipSuccess && time_out) e = copy_sync(ctx, time_out, d_time, sizeof(double) * n_tf, hipMemcpyDeviceToHost);
  if (e == hipSuccess && fills_out)
    e = copy_sync(ctx, fills_out, d_fills, sizeof(int32_t) * n_tf, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return cleanup(hip_fail(ctx, e, "download delivery results"));
  return cleanup(PMC_OK);
}
