/*
 * FP64 reference (oracle) for the condensed-history proton dose engine.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this library: only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code with the HIP implementation;
 * the only common ground is the seeded input generator and the written
 * specification of the transport model.
 *
 * Units at this interface: mm and MeV (as in the product's C ABI).  Inside:
 * cm, g/cm^3, MeV.
 */
#ifndef PMC_ORACLE_H
#define PMC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  const int16_t *hu;   /* nx*ny*nz, x fastest */
  const uint8_t *mask; /* nullable; 0 = outside the external contour (vacuum) */
  int32_t nx, ny, nz;
  double spacing_mm[3];
  double origin_mm[3]; /* corner of voxel (0,0,0) */
  const double *calib_hu, *calib_rho, *calib_rsp;
  int32_t n_nodes;
} orc_phase;

typedef struct {
  double isocentre_mm[3];
  double direction[3];
  double bev_u[3];
} orc_field;

typedef struct {
  double energy_MeV, x_mm, y_mm, sigma_mm, weight;
  int32_t phase, field;
} orc_spot;

/* physics switches (pin tests); the draw schedule never depends on them */
enum {
  ORC_NO_STRAGGLING = 1,
  ORC_NO_MCS = 2,
  ORC_NO_DELTA = 4,
  ORC_NO_NUCLEAR = 8,
  ORC_FROZEN = 16 /* energy never changes (no continuous loss; delta energy is
                     tallied but not removed from the proton) */
};

enum { ORC_CAUSE_STOP = 0, ORC_CAUSE_GEO = 1, ORC_CAUSE_DELTA = 2, ORC_CAUSE_NUCLEAR = 3, ORC_CAUSE_PHYS = 4 };
enum { ORC_FATE_ALIVE = 0, ORC_FATE_STOPPED = 1, ORC_FATE_ESCAPED = 2, ORC_FATE_NUCLEAR = 3, ORC_FATE_MISSED = 4 };

typedef struct {
  /* 128-bit unsigned totals, in units of 2^-32 MeV, as (lo, hi) words */
  uint64_t incident[2], deposited[2], escaped[2], nuclear[2], cutoff[2];
  uint64_t histories, steps, delta_events, nuclear_events, escapes, misses;
} orc_balance;

typedef struct {
  int32_t cause;   /* step-limiting cause (ORC_CAUSE_*), -1 for the source record */
  int32_t voxel;   /* linear voxel index where the step took place */
  int32_t fate;    /* ORC_FATE_* after this step */
  uint32_t block;  /* next unused Philox block index after this step */
  double s;        /* step length, cm */
  double E;        /* kinetic energy after the step and its events, MeV */
  double r[3];     /* position after the step, cm, relative to the grid corner */
  double w[3];     /* direction after the step */
  double n_delta, n_nuc, l_acc;
  int64_t dep;     /* energy tallied in `voxel` by this step, 2^-32 MeV units */
  double t_delta;  /* energy of the delta ray produced at the step end (0 if none) */
  double margin;   /* smallest relative gap of a decision taken in this step (which
                      axis or cause limits it, clamps, cutoffs, delta acceptance):
                      where another implementation, equal to rounding, may decide
                      otherwise */
} orc_trace_rec;

typedef struct {
  double e[1024], R[1024], mu_delta[1024], omega2[1024];
  double lnE0, dlnE;
} orc_tables;

/* Tables of the transport model (restricted range, hard-delta coefficient,
 * soft-straggling coefficient) on the 1024-node log-energy grid. */
void orc_build_tables(orc_tables *t);

/* Analytic per-energy quantities (MeV cm^2/g, cm^2/g, MeV^2 cm^2/g). */
double orc_stopping_unrestricted(double E);
double orc_stopping_restricted(double E);
double orc_mu_delta(double E);
double orc_omega2(double E);
double orc_highland_theta2(double E, double L_gcm2);
/* Table interpolation and inverse range (for tests). */
double orc_interp(const double *tab, double E);
double orc_range(double E);
double orc_range_inverse(double R);

/* Philox4x32-10 block function (Salmon et al., SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Delta-ray energy sampler used by the transport, run standalone: for the
 * given energy, draws n delta energies from blocks (b0.., h, s) of key. */
int orc_sample_delta(double E, uint32_t seed, uint32_t request_id, uint32_t h, uint32_t s,
                     int32_t n, double *T_out);

/* Largest-remainder split of n_hist histories over the spots whose phase is
 * listed; spots of other phases get 0.  Returns 0 or a negative error. */
int orc_split_histories(const orc_spot *spots, int64_t n_spots, const int32_t *phase_ids,
                        int32_t n_req_phases, uint64_t n_hist, int64_t *per_spot);

/* Full dose run.  tallies[i] (nx*ny*nz int64, zero-initialised by the
 * caller) receives the tally of phase_ids[i]; dose[i] (nullable) receives
 * Gy per history.  Phases are referenced by their index in `phases`. */
int orc_dose(const orc_phase *phases, int32_t n_phases, const orc_field *fields, int32_t n_fields,
             const orc_spot *spots, int64_t n_spots, const int32_t *phase_ids, int32_t n_req_phases,
             uint64_t seed, uint32_t request_id, uint64_t n_hist, uint32_t flags, int32_t n_threads,
             int64_t *const *tallies, double *const *dose, orc_balance *bal);

/* Same as orc_dose but only for the histories h of each spot (index within
 * the spot's share) with h_begin <= h < h_end and h % h_mod == h_rem: samples
 * of a full-size run, and the history batches of the statistical error. */
int orc_dose_subset(const orc_phase *phases, int32_t n_phases, const orc_field *fields,
                    int32_t n_fields, const orc_spot *spots, int64_t n_spots,
                    const int32_t *phase_ids, int32_t n_req_phases, uint64_t seed,
                    uint32_t request_id, uint64_t n_hist, uint32_t flags, int32_t n_threads,
                    uint32_t h_begin, uint32_t h_end, uint32_t h_mod, uint32_t h_rem,
                    int64_t *const *tallies, orc_balance *bal);

/* Same as orc_dose but only for the histories of spots s_begin <= s < s_end
 * (the split is still that of the whole request): the dose of a spot alone,
 * from which the per-spot influence matrix is defined. */
int orc_dose_spots(const orc_phase *phases, int32_t n_phases, const orc_field *fields,
                   int32_t n_fields, const orc_spot *spots, int64_t n_spots,
                   const int32_t *phase_ids, int32_t n_req_phases, uint64_t seed,
                   uint32_t request_id, uint64_t n_hist, uint32_t flags, int32_t n_threads,
                   int64_t s_begin, int64_t s_end, int64_t *const *tallies, orc_balance *bal);

/* orc_dose_spots restricted further to the histories h of each spot with
 * h % h_mod == h_rem (batches of the same histories for an error estimate). */
int orc_dose_spots_batch(const orc_phase *phases, int32_t n_phases, const orc_field *fields,
                         int32_t n_fields, const orc_spot *spots, int64_t n_spots,
                         const int32_t *phase_ids, int32_t n_req_phases, uint64_t seed,
                         uint32_t request_id, uint64_t n_hist, uint32_t flags, int32_t n_threads,
                         int64_t s_begin, int64_t s_end, uint32_t h_mod, uint32_t h_rem,
                         int64_t *const *tallies, orc_balance *bal);

/* Per-step trace of one history (spot index, history index within spot).
 * Returns the number of records written (<= max_rec) or a negative error. */
int orc_trace(const orc_phase *phase, const orc_field *fields, int32_t n_fields,
              const orc_spot *spots, int64_t n_spots, int64_t spot, uint32_t h, uint64_t seed,
              uint32_t request_id, uint32_t flags, orc_trace_rec *rec, int32_t max_rec);

/* Dose conversion of a tally: Gy per history (density from the calibration). */
int orc_convert(const orc_phase *phase, const int64_t *tally, uint64_t n_hist, double *dose,
                double *density);

#ifdef __cplusplus
}
#endif
#endif
