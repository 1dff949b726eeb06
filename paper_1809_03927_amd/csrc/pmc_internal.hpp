// Internal declarations of libpmc shared by its host and device translation
// units: data layouts that cross the host/device boundary and the launch
// descriptors of the kernels.  Not part of the public ABI (include/pmc.h).
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

namespace pmc {

constexpr int kMaxTargets = 64;  // phases per request (PMC_MAX_PHASES)

// Spot descriptor in the working precision R (float or double).
template <typename R> struct SpotDev {
  R c[3];          // central ray point: spot position on the BEV plane, cm, grid-relative
  R u[3];          // BEV axis u (unit)
  R v[3];          // BEV axis v = w x u
  R w[3];          // beam direction (unit)
  R sigma;         // lateral sigma, cm
  R E;             // energy, MeV
  int32_t target;  // tally slot of the request
  int32_t pad;
};

// One tally target = one phase of a request.
struct TargetDev {
  const int16_t *hu;
  const uint8_t *mask;  // nullable
  unsigned long long *tally;
  int32_t nx, ny, nz, lut;  // lut: index of this phase's 4096-entry LUT in the launch's LUT array
  double d[3];              // voxel size, cm
};
static_assert(sizeof(TargetDev) == 64, "TargetDev layout");

// A run of histories of one spot for the persistent engine.
struct WorkItem {
  int32_t spot;
  uint32_t h_begin;
  uint32_t h_count;
  uint32_t pad;
};

// Voxel box of one spot in an influence calculation: box-local entry
// (x, y, z) -> offset + x + n[0] (y + n[1] z) of the box scratch; n = 0 for
// spots without histories.
struct BoxDev {
  int32_t lo[3];
  int32_t n[3];
  long long offset;  // first entry, a multiple of kTile
  double n_hist;     // histories of the spot
  double pad;
};
static_assert(sizeof(BoxDev) == 48, "BoxDev layout");

// Core box of one spot for the block engine: voxels lo + [0, n) of the
// spot's phase grid, whose deposits a block accumulates in LDS while it runs
// the spot's histories; n[0] n[1] n[2] <= the launch's core capacity (n = 0:
// no core, every deposit goes to the phase tally).
struct CoreDev {
  int32_t lo[3];
  int32_t n[3];
  int32_t pad[2];
};

// Core of one spot for the block engine: slices d = j0 + j (0 <= j < n_sl)
// of the grid axis d closest to the beam, each with a window of wa x we
// voxels across (axes a = (d + 1) % 3 and e = (d + 2) % 3) whose corner
// follows the beam axis: corner_i(j) = clamp((A[i] + B[i] j) >> 16,
// amin[i], amax[i]) along a (i = 0) and e (i = 1), inside the grid (phase
// tallies) or the spot's box (influence calculations).  Voxel
// (corner_0(j) + x, corner_1(j) + y) of slice j is core entry
// j wa we + x + wa y.  n_sl = 0: no core.
struct SliceCore {
  int32_t d, j0, n_sl, wa, we;
  int32_t A[2], B[2];
  int32_t amin[2], amax[2];
  int32_t pad[3];
};
static_assert(sizeof(SliceCore) == 64, "SliceCore layout");

constexpr int kTile = 1024;  // box entries per compaction tile (256 threads x 4)

struct TraceRec {  // identical layout to pmc_trace_rec
  int32_t cause, voxel, fate;
  uint32_t block;
  double s, E, r[3], w[3], n_delta, n_nuc, l_acc;
  long long dep;
  double t_delta;
};

struct PlainLaunch {
  const void *spots;          // SpotDev<R>[n_spots]
  const int32_t *spot_ids;    // spots of this phase with histories, in spot order
  const long long *first;     // n_list + 1 prefix offsets of their histories
  int32_t n_list;
  long long n_hist;
  TargetDev target;
  const void *lut;            // R2[4096] of this phase
  const void *tab;            // R4[1024]
  double l2e0, inv_dl2, dl2;
  uint32_t k0, k1, flags;
  int block;
  bool lut_lds;
  unsigned long long *counters;
};

struct PersistentLaunch {
  const void *spots;
  const WorkItem *items;
  int32_t n_items;
  const TargetDev *targets;
  int32_t n_targets;
  const void *luts;           // R2[4096 * n_luts]
  const void *tab;
  double l2e0, inv_dl2, dl2;
  uint32_t k0, k1, flags;
  int32_t refill_min;
  int block;
  unsigned grid;
  bool lut_lds;
  unsigned long long *cursor;    // work-queue cursor, zero before the launch
  unsigned long long *counters;
  // influence calculations (boxes != nullptr): each spot tallies into its
  // box of `box_tally`, entry offset - box_bias
  const BoxDev *boxes = nullptr;
  unsigned long long *box_tally = nullptr;
  long long box_bias = 0;
  // host-visible flag set to 1 once every work item has been taken (nullable)
  unsigned int *drained = nullptr;
  // block engine (slices or cores != nullptr): one block per work item, LDS
  // room for core_cap tally entries per block; the core of each spot: its
  // slices, or for influence calculations whose cores are all straight (beams
  // along a grid axis) the same cores as windows of the boxes
  const SliceCore *slices = nullptr;
  bool slanted = false;  // some slice core follows an oblique beam
  const CoreDev *cores = nullptr;
  int32_t core_cap = 0;
  // block engine, measurement: the address of each lane's global atomics,
  // entry n of lane g at log[n * lanes + g] for n < log_cap, and each lane's
  // count of global atomics in log_count[g] (lanes = grid x kCoreBlock)
  unsigned long long *log = nullptr;
  uint32_t log_cap = 0;
  uint32_t *log_count = nullptr;
};

// Fixed LDS of a block-engine block (tables, the LUT when it is in LDS,
// counter reduction, item state); the core tally follows it.
size_t core_fixed_lds(bool lut_lds);
constexpr int kCoreBlock = 1024;  // threads per block-engine block

// Compaction of the box tallies of spots [0, n_spots) of a batch into CSR
// rows (voxel, Gy per history), voxels at or above rel_threshold x the
// spot's maximum of tally / density.
struct InfluenceLaunch {
  const long long *box_tally;   // batch scratch (entry 0 = box offset box_bias)
  const BoxDev *boxes;          // the batch's spots
  const long long *tile_first;  // n_spots + 1 tile prefix of the batch
  int32_t n_spots;
  long long n_tiles;
  long long box_bias;
  const int16_t *hu;
  const uint8_t *mask;
  const void *lut64;            // double2[4096]
  int32_t nx, ny;
  double vol_cm3;
  double rel_threshold;
  unsigned long long *spot_max;  // n_spots words (bits of the maximum, >= 0)
  unsigned long long *dep_sum;   // 2 words: 128-bit sum of the batch's tallies
  uint32_t *tile_count;          // n_tiles: entries with energy (zero before the passes)
  uint32_t *tile_keep;           // n_tiles: entries kept (zero before the passes)
  unsigned long long *tile_off;  // n_tiles: exclusive offsets within their chunk of kTile tiles
  unsigned long long *chunk_off; // n_chunks + 1: exclusive chunk offsets, last = batch total
  long long nnz_base;            // CSR entries before this batch
  int64_t *row_ptr;              // CSR row pointers of the batch's spots (n_spots entries)
  int32_t *voxel;
  float *value;
};

// Deformation vector field on the device (App. B): grid points i + n[0] (j +
// n[1] k) at start + i sp[0] u + j sp[1] v + k sp[2] w, translations delta
// (3 doubles per point, same order).
// DVF grid box (geometry only): the report mask tests points against it.
struct DvfBox {
  int32_t n[3];
  double start[3], sp[3];
  double u[3], v[3], w[3];
};

struct DvfDev {
  int32_t n[3];
  double start[3], sp[3];
  double u[3], v[3], w[3];
  const double *delta;
  int32_t has_pre, has_post;  // rigid matrices of Eq. (7) (rows 0..2 of 4x4)
  double pre[12], post[12];
};

// Energy/mass push of one source phase into the reference accumulators.
struct EmtmPush {
  const int16_t *hu;
  const uint8_t *mask;       // nullable
  const double *lut64;       // (rho, rsp) per HU -1024..3071
  const long long *tally;
  int32_t nx, ny, nz;
  double org[3], sp[3];      // source grid, mm
  DvfDev dvf;                // source -> reference
  int32_t rnx, rny, rnz;
  double rorg[3], rsp[3];    // reference grid, mm
  double rinv[3];            // 1 / rsp, rounded to nearest
  int32_t n_sub;
  int32_t aligned;           // DVF row (1,0,0) and column (0,1,0): per-axis grid coordinates
  unsigned long long *e_hi, *e_lo, *mass;  // per reference voxel
};

// dose_i += (e_hi 2^32 + e_lo) MeV_to_J / (mass vol 1e-3 n_hist) where mass > 0.
struct EmtmRatio {
  const unsigned long long *e_hi, *e_lo, *mass;
  double *dose;
  long long nvox;
  double vol_cm3, n_hist;
};

// Zero the dose (and clear the mask) outside the grid box of any of up to
// kMaskDvfs DVFs; `first` writes the mask, later passes only clear it.
constexpr int kMaskDvfs = 16;
struct EmtmMask {
  DvfBox dvfs[kMaskDvfs];
  int32_t n_dvf;
  int32_t first;
  int32_t nx, ny, nz;
  double org[3], sp[3];
  double *dose;
  uint8_t *mask_out;  // nullable
};

// Dose interpolation of one source phase (Eq. (3)): dose_i += average over
// the subvoxel centres of reference voxel i of the source dose sampled at
// their images under the reference-to-source DVF.
struct DimPull {
  int32_t nx, ny, nz;
  double org[3], sp[3];      // reference grid, mm
  DvfDev dvf;                // reference -> source
  int32_t snx, sny, snz;
  double sorg[3], ssp[3];    // source grid, mm
  const double *sdose;       // source dose per voxel (Gy per history)
  int32_t n_sub;
  int32_t aligned;           // as EmtmPush
  double *dose;
};

// Beam-delivery simulation (Sec. 2.B, App. A): one thread per (trial, field).
constexpr int kSyncParams = 9;
struct DeliverySpot {
  double e, x, y, mu;        // energy (MeV), BEV position (mm), MU
};
struct DeliveryLaunch {
  const DeliverySpot *spots; // grouped by field, plan order within a field
  const int32_t *fstart;     // n_fields + 1 offsets into spots
  const int64_t *index;      // plan index of each grouped spot
  int64_t n_spots;
  int32_t n_fields, n_trials, n_phases, start_phase, period_min, period_max, gate_lo, gate_hi;
  double period_s, period_sd_s, max_mu;
  double central[kSyncParams], sd[kSyncParams];
  uint32_t seed;
  double *mu;                // [trial][plan spot][phase], zeroed by the caller
  double *time;              // [trial][field], s
  int32_t *fills;            // [trial][field]
  int32_t *status;           // 1 if a thread stopped at its iteration cap
  int32_t layer_cap;         // layers of at most this many spots are staged in LDS
};
hipError_t launch_delivery(const DeliveryLaunch &a, hipStream_t st);

hipError_t launch_emtm_push(const EmtmPush &a, hipStream_t st);
hipError_t launch_dim_pull(const DimPull &a, hipStream_t st);
// Eqs. (8), (7) at every grid point; outputs nullable (device memory)
hipError_t launch_dvf_points(const DvfDev &d, double *x0, double *rf, hipStream_t st);
hipError_t launch_emtm_ratio(const EmtmRatio &a, hipStream_t st);
hipError_t launch_emtm_mask(const EmtmMask &a, hipStream_t st);

hipError_t launch_influence_reduce(const InfluenceLaunch &a, hipStream_t st);  // max, sum, count, scan
hipError_t launch_influence_write(const InfluenceLaunch &a, hipStream_t st);   // rows and entries, then clears the tiles with energy

struct TraceLaunch {
  const void *spot;  // host pointer to one SpotDev<R> (passed by value)
  int32_t spot_index;
  uint32_t h;
  TargetDev target;
  const void *lut, *tab;
  double l2e0, inv_dl2, dl2;
  uint32_t k0, k1, flags;
  void *rec;
  int32_t max_rec;
  int32_t *n_rec;
};

hipError_t launch_plain(const PlainLaunch &a, bool fp64, hipStream_t st);
hipError_t launch_persistent(const PersistentLaunch &a, bool fp64, hipStream_t st);
int persistent_blocks_per_cu(const PersistentLaunch &a, bool fp64);
hipError_t launch_trace(const TraceLaunch &a, bool fp64, hipStream_t st);
hipError_t launch_convert(const long long *tally, const int16_t *hu, const uint8_t *mask,
                          const void *lut64, long long nvox, double vol_cm3, double n_hist,
                          double *dose, double *density, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long *p, long long n, unsigned long long value,
                           hipStream_t st);
hipError_t launch_atomic_replay(const unsigned long long *log, uint32_t log_cap, const uint32_t *log_count,
                                uint32_t n_lanes, hipStream_t st);

// ---- the no-allocation entry point's scratch --------------------------------
// A file-scope device array of kNoAllocBytes per device (request data and
// the work-queue cursor of pmc_dose_device_noalloc), plus a pinned host
// staging buffer of the same size and an event marking the end of the last
// upload from it.  Set up once per device by noalloc_setup (with that device
// current: pmc_create calls it); everything stays until the process ends.
constexpr size_t kNoAllocBytes = size_t(8) << 20;
struct NoAlloc {
  unsigned char *dev = nullptr;   // address of the device array on this device
  unsigned char *host = nullptr;  // pinned staging
  hipEvent_t uploaded = nullptr;  // recorded after each upload from `host`
};
hipError_t noalloc_setup(int device, NoAlloc **out);

// ---- physics tables (host, FP64) -------------------------------------------
constexpr int kTableNodes = 1024;

struct Tables {
  double lnE[kTableNodes];
  double range[kTableNodes];    // restricted CSDA range, g/cm^2 of water
  double mu_delta[kTableNodes]; // hard-delta production coefficient, cm^2/g
  double omega2[kTableNodes];   // soft straggling variance, MeV^2 cm^2/g
  double l2e0, dl2;             // log2 E of node 0 and log2 spacing
};

void build_tables(Tables *t);

}  // namespace pmc
