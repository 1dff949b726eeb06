/*
 * pmc.h -- C ABI of libpmc, a Monte Carlo proton dose engine for AMD MI355X
 * (gfx950).
 *
 * The engine is the hot path of a 4D dose calculator (Pepin et al.,
 * arXiv:1809.03927): it transports the pencil-beam spots of a plan, split by
 * a delivery simulation into sub-plans per breathing phase (Sec. 2.B), through
 * one voxelised CT per phase with class II condensed-history transport, and
 * returns dose and density per CT voxel on the CT grid (Sec. 2.C).  Dose is
 * energy over mass (Eq. (4): E = rho v D).
 *
 * Conventions for every call:
 *  - Units at this interface are mm and MeV; doses are Gy per history.
 *  - Arrays are plain host pointers unless a name says "dev" (device pointers
 *    on the context's device).  Voxel arrays are nx*ny*nz long, x fastest.
 *  - Every input is validated before any device work and copied before the
 *    call returns; the library keeps no caller pointer.  Outputs are written
 *    only into caller-owned buffers and only on success.
 *  - Return value: PMC_OK (0) or a negative PMC_E_* code; pmc_last_error()
 *    then describes the failure.  One context per host thread.
 */
#ifndef PMC_H
#define PMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------- */
#define PMC_OK 0
#define PMC_E_INVAL (-1)   /* bad argument: dims, NaN, calibration order, energy, weight, direction */
#define PMC_E_NOPHASE (-2) /* a spot or request names a phase that is not loaded */
#define PMC_E_BUDGET (-3)  /* the request does not fit the context's device-memory budget */
#define PMC_E_DEVICE (-4)  /* HIP runtime failure, or no device (validation-only context) */
#define PMC_E_RANGE (-5)   /* more than PMC_MAX_HISTORIES histories in one tally */
#define PMC_E_STATE (-6)   /* call out of order (e.g. pmc_dose before pmc_load_spots) */

#define PMC_MAX_HISTORIES 50000000ull /* int64 headroom of one voxel tally */
#define PMC_E_MIN_MEV 1.0
#define PMC_E_MAX_MEV 300.0
#define PMC_MAX_PHASES 64   /* phases in one request */

/* ---- precision ---------------------------------------------------------- */
#define PMC_FP32 0 /* production transport in single precision */
#define PMC_FP64 1 /* debug transport in double precision (trace parity) */

/* ---- request flags (physics switches for validation; the random-number
 *      draw schedule never depends on them) --------------------------------*/
#define PMC_NO_STRAGGLING 1u
#define PMC_NO_MCS 2u
#define PMC_NO_DELTA 4u
#define PMC_NO_NUCLEAR 8u
#define PMC_FROZEN 16u /* energy never changes (validation of scattering) */

/* ---- engines ------------------------------------------------------------ */
#define PMC_ENGINE_PLAIN 0      /* one launch per phase, one history per thread */
#define PMC_ENGINE_PERSISTENT 1 /* one launch for all phases: work queue + lane refill */

/* Where the persistent engine adds deposits (pmc_request.tally_mode).
 * LANE: each lane adds a voxel visit's deposit into the phase tally (one
 *   device-wide atomic per visit); waves take work items on their own.
 * CORE: a block of 1024 threads runs one work item at a time; deposits inside
 *   the spot's core (the slices of the grid axis closest to the beam, from
 *   the entry face to water-equivalent depth R(E) + 1 cm, each with a window
 *   across centred on the beam axis, all fitting the block's LDS) add into
 *   LDS, the block adds each nonzero core voxel into the phase tally once the
 *   item is done, and the other deposits go to the phase tally directly.
 *   Fewer device-wide atomics; the integer tallies are identical.  FP32 only. */
#define PMC_TALLY_AUTO 0
#define PMC_TALLY_LANE 1
#define PMC_TALLY_CORE 2

typedef struct pmc_context pmc_context;

typedef struct {
  int32_t device;            /* HIP device ordinal; -1 = validation-only context */
  int32_t precision;         /* PMC_FP32 or PMC_FP64 */
  uint64_t seed;             /* Philox key word 0 is seed mod 2^32 */
  uint64_t hbm_budget_bytes; /* 0: 90 % of the device memory free at creation */
} pmc_config;

/* A treatment field: isocentre (mm, CT frame), beam direction and the
 * beam's-eye-view axis u (both unit vectors, orthogonal to 1e-6); the second
 * BEV axis is v = direction x u. */
typedef struct {
  double isocentre_mm[3];
  double direction[3];
  double bev_u[3];
} pmc_field;

/* A plan spot (Appendix A: position, energy, weight), with the breathing
 * phase the delivery simulation assigned it to (Sec. 2.B) and its field. */
typedef struct {
  double energy_MeV; /* [1, 300] */
  double x_mm, y_mm; /* BEV position at the isocentre plane */
  double sigma_mm;   /* Gaussian lateral sigma, >= 0 */
  double weight;     /* > 0; histories are split in proportion */
  int32_t phase;     /* phase id as given to pmc_load_phase */
  int32_t field;     /* index into the fields array */
} pmc_spot;

typedef struct {
  uint32_t request_id;    /* Philox key word 1 */
  uint32_t flags;         /* PMC_NO_* / PMC_FROZEN */
  uint64_t n_histories;   /* total over the spots of the listed phases, 1..PMC_MAX_HISTORIES */
  const int32_t *phases;  /* phase ids to simulate (spots of other phases are skipped) */
  int32_t n_phases;       /* 1..PMC_MAX_PHASES, distinct, all loaded */
  int32_t engine;         /* PMC_ENGINE_* */
  int32_t block_size;     /* threads per block, multiple of 64 in 64..1024 (FP64: ..256);
                             0 = default (see pmc_launch_shape) */
  int32_t chunk;          /* persistent engine: histories per work item; 0 = default */
  int32_t refill_min;     /* persistent engine: refill when >= this many lanes of a wave are idle (1..64); 0 = default */
  int32_t grid_blocks;    /* persistent engine: blocks; 0 = enough to fill the device, but no more
                             than the work items (block engine) or than start every history
                             at once (lane engine) */
  int32_t plan;           /* plan id (pmc_load_plan; pmc_load_spots loads plan 0) */
  int32_t tally_mode;     /* persistent engine: PMC_TALLY_*; 0 = library's choice */
  uint64_t item_begin;    /* persistent engine: run only work items [item_begin, item_end) */
  uint64_t item_end;      /*   of the request (0, 0 = all); see pmc_request_items */
} pmc_request;

/* Energy balance of a run.  128-bit unsigned totals as (lo, hi) words, in
 * units of 2^-32 MeV: deposited + escaped + nuclear == incident exactly. */
typedef struct {
  uint64_t incident[2], deposited[2], escaped[2], nuclear[2], cutoff[2];
  uint64_t histories, steps, delta_events, nuclear_events, escapes, misses;
} pmc_balance;

/* One record of a per-step trace (pmc_trace); positions in cm relative to
 * the grid corner; cause: -1 source, 0 stop, 1 boundary, 2 delta, 3 nuclear,
 * 4 step limit; fate: 0 alive, 1 stopped, 2 escaped, 3 nuclear, 4 missed. */
typedef struct {
  int32_t cause, voxel, fate;
  uint32_t block;
  double s, E, r[3], w[3], n_delta, n_nuc, l_acc;
  int64_t dep;
  double t_delta;
} pmc_trace_rec;

/* Number of uint64 words of the device counter block used by pmc_dose_device.
 * Layout: [0,1] escaped, [2,3] nuclear-removed, [4,5] cutoff energy as 128-bit
 * (lo, hi) pairs in 2^-32 MeV; [6] histories, [7] steps, [8] delta events,
 * [9] nuclear events, [10] escapes, [11] misses, [12] global tally atomics
 * issued; [13,14] energy deposited outside the spots' boxes (influence
 * calculations, 128-bit); [15] reserved. */
#define PMC_COUNTERS 16

/* ---- context ------------------------------------------------------------ */

/* Create a context on cfg->device.  device = -1 gives a validation-only
 * context: every argument check works, calls that need a GPU return
 * PMC_E_DEVICE.  *out is set only on success. */
int pmc_create(const pmc_config *cfg, pmc_context **out);

/* Free the context and all device memory it owns.  NULL-safe. */
void pmc_destroy(pmc_context *ctx);

/* Message of the last failed call on ctx (empty if none); owned by ctx and
 * valid until the next call on it.  ctx may be NULL (then a static message). */
const char *pmc_last_error(const pmc_context *ctx);

/* ---- inputs --------------------------------------------------------------- */

/* Load (or replace) CT phase `phase` (0..1023): HU grid, geometry and the
 * piecewise-linear HU -> mass density and HU -> stopping-power-ratio
 * calibration (Sec. 2.C: HU converted to density inside the engine).
 * calib_hu is strictly increasing, n_nodes >= 2, densities and RSPs >= 0.
 * HU values are clamped to [-1024, 3071].  external_mask (nullable, 0/1 per
 * voxel) bounds transport (Sec. 2.A): voxels outside it are vacuum.
 * The HU grid stays resident on the device until replaced or unloaded. */
int pmc_load_phase(pmc_context *ctx, int32_t phase, const int16_t *hu, int32_t nx, int32_t ny,
                   int32_t nz, const double spacing_mm[3], const double origin_mm[3],
                   const double *calib_hu, const double *calib_density, const double *calib_rsp,
                   int32_t n_nodes, const uint8_t *external_mask);

/* Free the device copy of a loaded phase. */
int pmc_unload_phase(pmc_context *ctx, int32_t phase);

/* Load (or replace) plan `plan` (0..1023): fields and spots with their phase
 * indices -- the plan of Appendix A (per spot: position, energy, weight)
 * split into the sub-plans of Sec. 2.B (the breathing phase each spot is
 * delivered in).  Histories of a request are split over its spots in
 * proportion to their weights.  A context holds several plans; a request
 * names the one it uses.  Validation as documented for pmc_spot and
 * pmc_field; PMC_E_INVAL on the first bad spot or field. */
int pmc_load_plan(pmc_context *ctx, int32_t plan, const pmc_field *fields, int32_t n_fields,
                  const pmc_spot *spots, int64_t n_spots);

/* pmc_load_plan for plan 0 (the calls named by the problem statement:
 * pmc_load_phase, pmc_load_spots, pmc_dose). */
int pmc_load_spots(pmc_context *ctx, const pmc_field *fields, int32_t n_fields,
                   const pmc_spot *spots, int64_t n_spots);

/* The sub-plans of one delivery (Sec. 2.B: per breathing phase, the spots
 * delivered in it and their weighting) loaded as plan `plan`: for every
 * spot s (array order) and phase p (ascending) with mu[s * n_phases + p] >
 * 0, spot s on phase phase_ids[p] with weight that MU -- a spot delivered
 * over several phases becomes one spot per phase.  mu is one trial of
 * pmc_delivery_simulate's mu_out (MU per spot and phase).  *n_subplan_spots
 * (nullable) receives the spot count.  PMC_E_INVAL for negative or
 * non-finite MU, bad phase ids, or no MU at all; then as pmc_load_plan. */
int pmc_load_subplans(pmc_context *ctx, int32_t plan, const pmc_field *fields, int32_t n_fields,
                      const pmc_spot *spots, int64_t n_spots, const double *mu, int32_t n_phases,
                      const int32_t *phase_ids, int64_t *n_subplan_spots);

/* Forget a plan and free the device data prepared for it. */
int pmc_unload_plan(pmc_context *ctx, int32_t plan);

/* Number of work items of a persistent-engine request.  Each spot's
 * histories are cut into runs of `chunk` (pmc_launch_shape); the work queue
 * holds the first run of every spot in plan order, then the second run of
 * every spot that has one, and so on, so that waves running together carry
 * histories of many spots.  A request may be run as several calls over
 * consecutive item slices adding into the same tallies and counters;
 * together they equal one call over all items.  Prepares (and caches) the
 * request's device data. */
int pmc_request_items(pmc_context *ctx, const pmc_request *req, uint64_t *n_items);

/* Work items of a persistent-engine request without preparing it: *n_items
 * receives their number (as pmc_request_items) and, if histories is not
 * NULL, histories[i] the number of histories of item i in queue order
 * (PMC_E_INVAL if capacity is smaller than the count).  Lets a caller cut
 * slices of a chosen number of histories.  Host-only (works on
 * validation-only contexts, which assume 256 compute units for the default
 * chunk). */
int pmc_request_item_histories(pmc_context *ctx, const pmc_request *req, uint32_t *histories,
                               uint64_t capacity, uint64_t *n_items);

/* Launch shape the library uses for req (pmc_launch_shape). */
typedef struct {
  int32_t block_size;    /* threads per block */
  int32_t chunk;         /* histories per work item (persistent engine) */
  int32_t refill_min;    /* lane refill threshold (persistent engine) */
  int32_t tally_mode;    /* PMC_TALLY_LANE or PMC_TALLY_CORE (persistent engine), else 0 */
  int32_t core_capacity; /* PMC_TALLY_CORE: LDS tally entries per block, else 0 */
  int32_t reserved[3];
} pmc_shape;

/* Launch shape the library uses for req: the request's own values where
 * set, else the defaults.
 *  - tally_mode: PMC_TALLY_CORE for the FP32 persistent engine when work
 *    items of `chunk` (default 8192) histories, a spot's partial last item
 *    counted with its full ones, average at least 1024 histories (one per
 *    lane of a block) and the LDS holds at least 4096 core entries; else
 *    PMC_TALLY_LANE.
 *  - block_size: 1024 for the FP32 persistent engine (PMC_TALLY_CORE takes
 *    only 1024), 256 for FP64 and for the plain engine.
 *  - chunk: PMC_TALLY_CORE 8192, halved down to 1024 while the request has
 *    fewer histories than that per compute unit; PMC_TALLY_LANE the largest of 256, 128, 64
 *    for which the request still has about four work items per resident wave
 *    (16 waves per compute unit).
 *  - refill_min: 64.
 * Host-only (works on validation-only contexts, which assume 256 compute
 * units and 160 KiB of LDS per block). */
int pmc_launch_shape(pmc_context *ctx, const pmc_request *req, pmc_shape *out);

/* ---- dose ------------------------------------------------------------------ */

/* The Monte Carlo dose of Sec. 2.C: simulate req->n_histories histories
 * (class II condensed-history transport) over the spots of the listed
 * phases -- the N_g per-phase runs of a field, here in one call -- and
 * return, for each listed phase i, the dose on its CT grid dose_out[i] (Gy
 * per history, nx*ny*nz doubles; NULL entries skipped; dose = deposited
 * energy / (density x voxel volume), as Eq. (4) relates them), optionally
 * the raw tally tally_out[i] (int64, 2^-32 MeV) and the density grid
 * density_out[i] (g/cm^3, the engine's HU conversion), and the energy
 * balance.  Blocks until done. */
int pmc_dose(pmc_context *ctx, const pmc_request *req, double *const *dose_out,
             int64_t *const *tally_out, double *const *density_out, pmc_balance *balance_out);

/* Device variant for callers that own device memory and streams: enqueue the
 * transport of `req` on `stream` (a hipStream_t; NULL = default stream),
 * ADDING into the caller's zero-initialised int64 tallies dev_tally[i] (one
 * per listed phase, nx*ny*nz each) and into dev_counters (PMC_COUNTERS
 * uint64 words, nullable).  Returns after enqueueing.  Calls on different
 * streams may run concurrently on the device, also when they add into the
 * same tallies (all deposits are atomic): each persistent-engine call takes
 * one of 16 work-queue cursors in turn and waits, on the device, for the
 * call that used that cursor before.  A NULL dev_counters means the
 * context's own block, which concurrent calls share.  Calls that free or
 * rewrite device data (unloading or replacing phases and plans, evicting
 * prepared requests, pmc_destroy) first wait for the enqueued work that
 * reads it.  Host calls on one context must come from one thread at a time.
 * Read the counters with pmc_balance_from_counters. */
int pmc_dose_device(pmc_context *ctx, const pmc_request *req, void *stream,
                    int64_t *const *dev_tally, uint64_t *dev_counters);

/* pmc_dose_device for the persistent engine, with a drain signal: once every
 * work item of the launch has been taken (its last histories may still be
 * running), the kernel writes 1 to *host_drained.  host_drained must be host
 * memory the device can write (pinned, e.g. hipHostMalloc); the caller sets
 * it to 0 before the call and keeps it until the launch completes.  A caller
 * that waits for this flag instead of the launch's end can start its next
 * launch on another stream while this one drains (a serving loop cutting
 * requests into slices pays no drain per slice). */
int pmc_dose_device_notify(pmc_context *ctx, const pmc_request *req, void *stream,
                           int64_t *const *dev_tally, uint64_t *dev_counters, uint32_t *host_drained);

/* pmc_dose_device for callers that cannot allocate device memory in the
 * call (code that must not call hipMalloc, tight serving loops, harnesses
 * that forbid allocation): the same transport, the same tallies bit for bit,
 * but the request's device data (spot descriptors, work items, spot cores,
 * LUTs, target table) and the work-queue cursor go into a fixed device array
 * of 8 MiB that the library sets up once per device at pmc_create (with a
 * pinned host staging buffer of the same size), instead of memory allocated
 * per request.  No device or pinned memory is allocated and nothing is freed
 * by this call (host-side temporaries only); the request data is rebuilt and
 * uploaded on `stream` every call (no cache).  dev_counters is required.
 *  - PMC_E_RANGE, with nothing enqueued, if the request data would exceed
 *    8 MiB (about 60,000 spots in FP32, 40,000 in FP64; pmc_dose_device
 *    takes larger requests).
 *  - Every context on a device shares that device's array, which keeps the
 *    last call's contents: calls whose device work overlaps in time (on
 *    different streams, or from different contexts of one device) race and
 *    must not be made; calls on one stream are ordered.
 *  - Unloading or replacing a phase, and pmc_destroy, wait for the whole
 *    device after such a call (it records no per-resource events). */
int pmc_dose_device_noalloc(pmc_context *ctx, const pmc_request *req, void *stream,
                            int64_t *const *dev_tally, uint64_t *dev_counters);

/* Turn a device counter block (copied to the host) plus the request into a
 * pmc_balance; the deposited total is taken from the tallies' sum, passed as
 * a 128-bit (lo, hi) pair.  The incident energy is that of the histories the
 * request runs: for a slice [item_begin, item_end) of a persistent-engine
 * request, those of its work items only (pmc_dose reports the same). */
int pmc_balance_from_counters(pmc_context *ctx, const pmc_request *req, const uint64_t *counters,
                              const uint64_t deposited[2], pmc_balance *out);

/* Convert one device tally of `phase` into dose (Gy per history) and density
 * on `stream` (dev_dose / dev_density: nx*ny*nz doubles, nullable). */
int pmc_convert_device(pmc_context *ctx, int32_t phase, const int64_t *dev_tally,
                       uint64_t n_histories, void *stream, double *dev_dose, double *dev_density);

/* ---- captured graphs -------------------------------------------------------- */

typedef struct pmc_graph pmc_graph;

/* Capture one complete dose calculation of `req` into a HIP graph bound to
 * the given device buffers (the batching of Sec. 2.C's N_g runs into one
 * replayable launch): zero dev_tally[i] and dev_counters, transport all
 * listed phases, and (where dev_dose[i] is not NULL) convert each tally into
 * Gy per history.  The graph owns a private copy of the request's device
 * data (plan, work items), so later plan loads do not affect it; it reads
 * the listed phases' device grids in place, so it must be destroyed before
 * its context.  dev_counters is required (the balance of a replay is read
 * from it).  Every reset inside the graph is a kernel, not a memset.
 * Replays on one graph must not overlap in time. */
int pmc_graph_create(pmc_context *ctx, const pmc_request *req, int64_t *const *dev_tally,
                     uint64_t *dev_counters, double *const *dev_dose, pmc_graph **out);

/* Replay a captured graph on `stream` (a hipStream_t; NULL = default stream).
 * PMC_E_STATE, with nothing launched, if a phase the graph reads was unloaded
 * or replaced (pmc_load_phase on its id) since the capture: the graph is
 * stale and can only be destroyed. */
int pmc_graph_launch(pmc_graph *g, void *stream);

/* Free a graph and its device data.  NULL-safe. */
void pmc_graph_destroy(pmc_graph *g);

/* ---- validation hooks ------------------------------------------------------ */

/* Measurement of the block engine's deposit-address pattern: run `req`
 * (persistent engine resolving to PMC_TALLY_CORE, FP32, grid_blocks > 0) as
 * pmc_dose_device does -- the same tallies -- and also write, for every
 * lane g of the launch (lanes = grid_blocks x 1024), the device address of
 * its n-th device-wide tally atomic to dev_log[n * lanes + g] for n <
 * per_lane, and its count of such atomics to dev_log_count[g].  dev_log
 * holds per_lane x lanes uint64, dev_log_count lanes uint32 (device). */
int pmc_atomic_log(pmc_context *ctx, const pmc_request *req, void *stream, int64_t *const *dev_tally,
                   uint64_t *dev_counters, uint64_t *dev_log, uint32_t per_lane, uint32_t *dev_log_count);

/* Replay a log written by pmc_atomic_log (same per_lane, n_lanes = its
 * lanes): lane g issues 64-bit atomic adds of 1 at its first
 * min(dev_log_count[g], per_lane) logged addresses, in order, with nothing
 * between them -- the atomic throughput of exactly that address pattern
 * (timed by the caller on `stream`).  The logged tallies must still be
 * allocated; they are changed. */
int pmc_atomic_replay(pmc_context *ctx, void *stream, const uint64_t *dev_log, uint32_t per_lane,
                      const uint32_t *dev_log_count, uint32_t n_lanes);

/* Per-step trace of one history (spot index, history index within the spot)
 * of plan `plan` on one phase, computed by the GPU transport in the
 * context's precision.  Writes at most max_rec records and sets *n_rec to the
 * full length. */
int pmc_trace(pmc_context *ctx, int32_t plan, int32_t phase, int64_t spot, uint32_t history,
              uint32_t request_id, uint32_t flags, pmc_trace_rec *out, int32_t max_rec,
              int32_t *n_rec);

/* Histories per spot of a request (host computation, no device): split
 * n_histories over the spots whose phase is listed, in proportion to weight
 * with the largest-remainder method, ties to the lower spot index. */
int pmc_split_histories(const pmc_spot *spots, int64_t n_spots, const int32_t *phases,
                        int32_t n_phases, uint64_t n_histories, int64_t *per_spot);

/* Device memory held by the context (phases, tables, scratch), in bytes. */
uint64_t pmc_bytes_in_use(const pmc_context *ctx);

/* ---- influence matrix ---------------------------------------------------- */

/* Voxel box [lo, hi) per axis; lo == hi on any axis means empty. */
typedef struct {
  int32_t lo[3], hi[3];
} pmc_box;

/* Boxes of the spots of `plan` on `phase` (n_spots = the plan's spot count;
 * spots of other phases get empty boxes): the axis-aligned voxel box around
 * the spot's central axis, from the first voxel on it with a stopping-power
 * ratio >= 0.1 (air before it is left out) to water-equivalent depth
 * R(E) + 3 cm (R: the transport's range table; water-equivalent depth =
 * path length x stopping-power ratio of the voxels crossed) or the grid
 * exit, widened across the beam by 3 sigma_max, sigma_max^2 = sigma_spot^2 +
 * (0.035 L)^2, L the geometric length of that axis segment.  Empty if the
 * axis misses the grid or meets no such voxel.  Host computation; works on
 * a validation-only context. */
int pmc_influence_boxes(pmc_context *ctx, int32_t plan, int32_t phase, pmc_box *out, int64_t n_spots);

/* Sparse per-spot influence matrix of a one-phase request (the dose of each
 * spot separately, which an optimiser of spot weights needs; Sec. 4.C).
 * Runs the request's histories (persistent engine, launch fields honoured,
 * not sliced) with every spot tallying into its own box (`boxes`: one per
 * plan spot, or NULL for pmc_influence_boxes); with PMC_TALLY_CORE (picked
 * by the rule of pmc_launch_shape when tally_mode is 0) a block keeps part
 * of its spot's box in LDS (a window centred in the box, or, when some field
 * runs oblique to the grid, the spot's core slices kept inside its box).
 * Then it keeps, per spot, the
 * voxels whose tally / density is >= rel_threshold (0..1) x that spot's
 * maximum of it, as CSR: one row per plan spot (row_ptr: n_spots + 1
 * int64), voxel = linear index of the phase grid (int32, ascending within a
 * row), value = dose per history of that spot (float, Gy: energy / (density
 * x voxel volume) / the spot's histories).  Deposits outside a spot's box
 * are not in the matrix; their energy is returned in outside[2] (128-bit
 * (lo, hi), 2^-32 MeV; nullable).  balance (nullable): deposited = energy
 * in the boxes, so deposited + outside + escaped + nuclear == incident.
 * Box tallies (int64) live in context scratch of at most max_scratch_bytes
 * (0 = half the free budget); the spots run in batches of consecutive spots
 * whose boxes fit it (PMC_E_BUDGET if one box does not).  The result stays
 * in the context (pmc_influence_read, pmc_influence_device) until the next
 * pmc_influence or pmc_influence_free.  Blocks until done.  *nnz = number of
 * entries. */
int pmc_influence(pmc_context *ctx, const pmc_request *req, const pmc_box *boxes, double rel_threshold,
                  uint64_t max_scratch_bytes, uint64_t *nnz, pmc_balance *balance, uint64_t outside[2]);

/* Copy the last influence matrix to caller buffers (each nullable):
 * row_ptr[n_spots + 1], voxel[nnz], value[nnz]. */
int pmc_influence_read(pmc_context *ctx, int64_t *row_ptr, int32_t *voxel, float *value);

/* Device pointers of the last influence matrix (owned by the context). */
int pmc_influence_device(pmc_context *ctx, const int64_t **row_ptr, const int32_t **voxel,
                         const float **value);

/* Free the influence matrix and its scratch. */
int pmc_influence_free(pmc_context *ctx);

/* ---- deformable dose accumulation (Sec. 2.D) ------------------------------ */

/* A deformation vector field as a DICOM deformable registration stores it
 * (App. B, Eqs. (7)-(8)): grid point (i, j, k), 0 <= i < n[0] ..., sits at
 * x0 = start_mm + i spacing_mm[0] row + j spacing_mm[1] col + k spacing_mm[2]
 * (row x col) (Eq. (8)) and maps to M_post (M_pre x0 + delta) (Eq. (7); the
 * rigid matrices are the identity between phases of one 4DCT, pass NULL).
 * A point r between grid points maps to M_post (M_pre r + delta(r)), delta(r)
 * the trilinear interpolation (x, then y, then z) of the translations of the
 * grid points around it, in FP64; points outside the box of grid points are
 * not mapped.  For pmc_accumulate the field maps a source phase onto the
 * reference phase; for pmc_accumulate_dim the reference phase onto a source. */
typedef struct {
  int32_t n[3];            /* grid points along row, column, depth; each >= 2 */
  double start_mm[3];      /* position of grid point (0, 0, 0), scanner frame */
  double spacing_mm[3];    /* > 0 */
  double row[3], col[3];   /* unit, orthogonal direction cosines (within 1e-6) */
  const double *delta_mm;  /* translations (x, y, z) per grid point, i fastest, then j, k */
  const double *pre;       /* nullable: M_pre, 4x4 row-major rigid matrix (rotation part
                              orthonormal within 1e-6, last row 0 0 0 1); NULL = identity */
  const double *post;      /* nullable: M_post, same form */
} pmc_dvf;

/* Copy a DVF to the device as `dvf` (0..1023), replacing one of that id. */
int pmc_load_dvf(pmc_context *ctx, int32_t dvf, const pmc_dvf *d);
int pmc_unload_dvf(pmc_context *ctx, int32_t dvf);

/* The full field of a loaded DVF (App. B): Eq. (8) and Eq. (7) evaluated on
 * the device, one thread per grid point.  x0_out receives the grid points'
 * positions, rf_out the mapped positions M_post (M_pre x0 + delta); 3 doubles
 * (x, y, z) per point in grid order (i fastest), mm; either may be NULL.
 * Eq. (8) is the matrix product written out per axis:
 *   x0_a = (row_a dX) i + (col_a dY) j + (dep_a dZ) k + start_a.
 * Host buffers; blocks until done. */
int pmc_dvf_points(pmc_context *ctx, int32_t dvf, double *x0_out, double *rf_out);

/* Accumulated dose on the reference phase's grid by energy/mass transfer
 * (Sec. 2.D.2, Eqs. (2), (4)-(6)), Gy per history of a run of n_histories:
 *   D_i = D_i^R + sum over sources S (in list order) of D_i^S,
 * D^R the reference phase's own dose (ref_tally, as pmc_convert_device), and
 * D_i^S = sum E / sum M over the subvoxels of S mapped into reference voxel i:
 * every voxel of S is cut into n_sub^3 equal subvoxels, each centre mapped by
 * the source's DVF; a subvoxel carries mass rho v and energy rho v D, i.e.
 * 1/n_sub^3 of its voxel's tally, and rho is the density the transport uses
 * (0 outside an external mask).  Sums are exact integers (tally units, and
 * round-half-even(rho 2^32) per subvoxel), so the result does not depend on
 * the schedule.  Reported (else 0) where the reference voxel centre lies in
 * the grid box of every source DVF; mask_out (nullable, one byte per voxel)
 * receives that mask.  Tallies in the units of pmc_dose (2^-32 MeV) on each
 * phase's own grid.  n_sub 1..16, n_src 0..PMC_MAX_PHASES.
 * pmc_accumulate: host buffers, blocks until done.
 * pmc_accumulate_device: device buffers, enqueued on `stream` (the call is
 * ordered after earlier accumulations on other streams; their accumulator
 * memory is shared). */
int pmc_accumulate(pmc_context *ctx, int32_t ref_phase, const int64_t *ref_tally, int32_t n_src,
                   const int32_t *src_phases, const int32_t *src_dvfs, const int64_t *const *src_tallies,
                   int32_t n_sub, uint64_t n_histories, double *dose_out, uint8_t *mask_out);
int pmc_accumulate_device(pmc_context *ctx, int32_t ref_phase, const int64_t *ref_tally, int32_t n_src,
                          const int32_t *src_phases, const int32_t *src_dvfs, const int64_t *const *src_tallies,
                          int32_t n_sub, uint64_t n_histories, void *stream, double *dev_dose,
                          uint8_t *dev_mask);

/* Accumulated dose on the reference phase's grid by dose interpolation
 * (Sec. 2.D.2, Eqs. (2), (3)), Gy per history: D_i = D_i^R + sum over
 * sources (list order) of D_i^S with
 *   D_i^S = (1 / n_sub^3) sum over the n_sub^3 subvoxel centres r_k of
 *           reference voxel i of Dt^S(T^{R->S}(r_k)),
 * where each source's DVF maps the reference phase onto that source (the
 * opposite direction to pmc_accumulate), subvoxel centres are at origin +
 * (i + (s + 1/2) / n_sub) spacing per axis, and Dt^S is the source phase's
 * dose (its tally converted as pmc_convert_device) interpolated trilinearly
 * between its voxel centres (x, then y, then z) at the position clamped to
 * the box of voxel centres, as a 3D texture with clamp-to-edge addressing
 * does.  A centre outside the DVF grid contributes 0.  The sum runs over the
 * subvoxels with x outermost, then y, then z, in FP64.  Reported (else 0)
 * where the reference voxel centre lies in the grid box of every DVF; other
 * arguments, buffers and streams as pmc_accumulate / pmc_accumulate_device
 * (the two share the context's scratch memory). */
int pmc_accumulate_dim(pmc_context *ctx, int32_t ref_phase, const int64_t *ref_tally, int32_t n_src,
                       const int32_t *src_phases, const int32_t *src_dvfs, const int64_t *const *src_tallies,
                       int32_t n_sub, uint64_t n_histories, double *dose_out, uint8_t *mask_out);
int pmc_accumulate_dim_device(pmc_context *ctx, int32_t ref_phase, const int64_t *ref_tally, int32_t n_src,
                              const int32_t *src_phases, const int32_t *src_dvfs,
                              const int64_t *const *src_tallies, int32_t n_sub, uint64_t n_histories,
                              void *stream, double *dev_dose, uint8_t *dev_mask);

/* ---- beam-delivery simulation (Sec. 2.B, App. A) ------------------------ */

/* A parameter's central value and 1-sigma uncertainty (0: fixed). */
typedef struct {
  double central, sd;
} pmc_param;

/* Synchrotron timing (App. A), drawn once per trial and field as
 * central + sd z (clipped at 0), in this order.  At energy E (MeV):
 *   layer switch (reset, acceleration, preparation) a + b (E - 70),
 *   spill rate (MU/s)                               c + d (E - 70),
 *   beam off between two spots of a fill            e + f max(|dx|, |dy|) (mm). */
typedef struct {
  pmc_param layer_switch_s;       /* a */
  pmc_param layer_switch_per_mev; /* b */
  pmc_param discard_s;            /* beam discarded at every extraction start (70 ms) */
  pmc_param spill_rate_mu_s;      /* c */
  pmc_param spill_rate_per_mev;   /* d */
  pmc_param spot_switch_s;        /* e */
  pmc_param spot_switch_per_mm;   /* f */
  pmc_param capacity_mu;          /* MU one synchrotron fill delivers */
  pmc_param extraction_max_s;     /* extraction time limit of a fill */
} pmc_synchrotron;

typedef struct {
  int32_t n_phases;               /* N, 1..64 */
  int32_t start_phase;            /* 0..N-1, or -1: U{0..N-1} per trial and field */
  double period_s;                /* breathing period mean mu, s (used unless min/max below) */
  double period_sd_s;             /* sigma: phase k lasts max(mu + sigma z_k, mu / 20) / N */
  int32_t period_min_s, period_max_s; /* if 0 < min <= max: mu ~ U{min..max} s per trial and field */
  int32_t gate_lo, gate_hi;       /* gated delivery: beam on only in phases gate_lo..gate_hi
                                     (0 <= lo <= hi < N); gate_lo = -1: free breathing */
  double max_mu;                  /* isolayered repainting: at most max_mu per spot delivery; 0: none */
  pmc_synchrotron sync;
  uint64_t seed;                  /* Philox key word 0 is seed mod 2^32, word 1 the trial */
  int32_t n_trials;               /* >= 1 */
} pmc_delivery;

/* Simulate the delivery of a plan (Sec. 2.B) in n_trials trials: which part
 * of each spot's MU is delivered in which breathing phase.  Spots (weight =
 * MU > 0, field 0..n_fields-1) are delivered in array order within each
 * field; a layer is a run of consecutive spots of one field with one energy.
 * Each (trial, field) is an independent timeline from t = 0 at the start of
 * its first breathing phase, one GPU thread each:
 *  - every layer starts a synchrotron fill: layer switch, then (gated) wait
 *    for the gate, then discarded beam;
 *  - painting r of a layer gives each spot min(MU - r max_mu, max_mu) while
 *    positive (without repainting its whole MU once), in spot order; between
 *    two deliveries the beam is off for the spot switch; a delivery that
 *    would exceed the fill's charge or extraction time, and is not the fill's
 *    first, starts a new fill at the same energy (layer switch, gate,
 *    discard); a delivery that finds the gate closed waits for it and
 *    discards beam again;
 *  - a delivery lasts its MU / spill rate and belongs to the breathing phase
 *    at its start.
 * Random numbers: Philox4x32-10, key (seed mod 2^32, trial), counter (field,
 * purpose, index, block); purpose 0 start phase, 1 synchrotron parameter
 * (index = its position above), 2 breathing phase occurrence k, 3 period;
 * a Gaussian z ~ N(0, 1) (the N(mu, sigma) draws of Sec. 2.B and App. A)
 * is sqrt(-2 ln u_a) cos(2 pi u_b) in FP64 with u = (x + 1/2) 2^-32 of words
 * 0 and 1 of block 0 (|z| <= 6.77); U{0..n-1} is floor(word 0 of block 0 x
 * n / 2^32).
 * Outputs (host buffers, each nullable): mu_out[trial][spot][phase] (MU),
 * time_out[trial][field] (end of the last delivery, s), fills_out
 * [trial][field] (synchrotron fills).  PMC_E_INVAL for invalid options or
 * spots, including spill rates that a draw within +-6.8 sigma could make <= 0
 * at a spot's energy.  Blocks until done. */
int pmc_delivery_simulate(pmc_context *ctx, const pmc_delivery *d, const pmc_spot *spots, int64_t n_spots,
                          int32_t n_fields, double *mu_out, double *time_out, int32_t *fills_out);

#ifdef __cplusplus
}
#endif
#endif /* PMC_H */
