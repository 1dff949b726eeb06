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
};

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
