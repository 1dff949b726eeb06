/*
 * FP64 reference (oracle) for the condensed-history proton dose engine.
 *
 * TEST INFRASTRUCTURE ONLY: used by tests, the smoke check and the benchmark's
 * CPU-baseline leg; never by the product path.  Plain, slow, obviously
 * correct: one history at a time, double precision throughout, no blocking,
 * no fusion.  Threads (pthreads) only split the list of histories; every
 * tally update is an integer add, so results do not depend on the number of
 * threads.
 *
 * What is computed, and where it comes from:
 *  - Sec. 2.C of the paper: a class II condensed-history proton transport
 *    whose dose grid is the CT grid, with HU converted to density inside the
 *    engine, returning dose and density per CT voxel.  The paper gives no
 *    further physics (its engine is described in its Refs. 33/34), so the
 *    model below is a textbook class II scheme; every choice where the paper
 *    is silent is listed as a reading in the design notes:
 *      * continuous loss from the restricted Bethe stopping power (energy
 *        transfers below T_cut), through the restricted CSDA range table;
 *      * hard delta rays above T_cut produced explicitly (free-electron
 *        spectrum for a spin-1/2 heavy projectile, cf. the PDG review
 *        "Passage of particles through matter") and absorbed locally;
 *      * Gaussian soft straggling with the Bohr-type variance of the
 *        restricted spectrum;
 *      * multiple Coulomb scattering with the Highland formula applied to the
 *        accumulated mass path ("telescoping"), a Rayleigh polar angle and a
 *        uniform azimuth;
 *      * nuclear removal with a constant mass attenuation above 10 MeV.
 *  - Eq. (4) of the paper: dose = energy / (density x volume); used for the
 *    dose conversion.
 *  - Footnote b of the paper (all GPU sampling from a library generator): here
 *    Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), keyed by
 *    (seed, request) with counter (block, history, spot, 0).
 */
#include "pmc_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------------- */
/* constants (CODATA / PDG)                                                */
/* ---------------------------------------------------------------------- */
#define ME 0.51099895          /* electron rest energy, MeV */
#define MP 938.27208816        /* proton rest energy, MeV */
#define KBETHE 0.307075        /* 4 pi N_A r_e^2 m_e c^2, MeV cm^2 / mol */
#define ZA 0.555087            /* water Z/A, mol / g */
#define IEXC 75.0e-6           /* water mean excitation energy, MeV */
#define X0W 36.08              /* water radiation length, g / cm^2 */
#define MEV_TO_J 1.602176634e-13
#define E_LO 1.0               /* transport cutoff and table floor, MeV */
#define E_HI 300.0             /* table ceiling, MeV */
#define T_CUT 0.1              /* delta-ray production threshold, MeV */
#define MU_N 0.0115            /* nuclear removal, cm^2 / g, for E >= E_N */
#define E_N 10.0
#define EPS_R 0.1              /* step limit: fraction of residual range */
#define S_FLOOR 0.01           /* step floor, cm water-equivalent */
#define NTAB 1024
#define HU_MIN (-1024)
#define HU_MAX 3071
#define MAX_STEPS (1 << 20)
#define TWO_PI 6.283185307179586476925286766559
#define Q_SCALE 4294967296.0   /* 2^32 */

typedef unsigned __int128 u128;

/* ---------------------------------------------------------------------- */
/* Philox4x32-10                                                           */
/* ---------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
    uint32_t y1 = (uint32_t)p1;
    uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
    uint32_t y3 = (uint32_t)p0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    k0 += 0x9E3779B9u; /* key schedule: golden ratio and sqrt(3)-1 words */
    k1 += 0xBB67AE85u;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* uniform in (0,1): (x + 1/2) 2^-32 */
static void draw4(const uint32_t key[2], uint32_t block, uint32_t h, uint32_t s, double u[4]) {
  uint32_t ctr[4] = {block, h, s, 0u}, x[4];
  orc_philox4x32_10(ctr, key, x);
  for (int k = 0; k < 4; ++k) u[k] = ((double)x[k] + 0.5) / Q_SCALE;
}

/* ---------------------------------------------------------------------- */
/* kinematics and stopping                                                 */
/* ---------------------------------------------------------------------- */
typedef struct { double beta2, b2g2, tmax, pbc; } kin_t;

static kin_t kinematics(double E) {
  kin_t k;
  double gamma = 1.0 + E / MP;
  k.b2g2 = gamma * gamma - 1.0;             /* (beta gamma)^2 */
  k.beta2 = 1.0 - 1.0 / (gamma * gamma);
  double r = ME / MP;
  k.tmax = 2.0 * ME * k.b2g2 / (1.0 + 2.0 * gamma * r + r * r);
  k.pbc = E * (E + 2.0 * MP) / (E + MP);    /* p beta c = (pc)^2 / (E_total) */
  return k;
}

double orc_stopping_unrestricted(double E) {
  kin_t k = kinematics(E);
  double arg = 2.0 * ME * k.b2g2 * k.tmax / (IEXC * IEXC);
  return KBETHE * ZA / k.beta2 * (0.5 * log(arg) - k.beta2);
}

double orc_stopping_restricted(double E) {
  kin_t k = kinematics(E);
  double tup = k.tmax < T_CUT ? k.tmax : T_CUT;
  double arg = 2.0 * ME * k.b2g2 * tup / (IEXC * IEXC);
  return KBETHE * ZA / k.beta2 * (0.5 * log(arg) - 0.5 * k.beta2 * (1.0 + tup / k.tmax));
}

double orc_mu_delta(double E) {
  kin_t k = kinematics(E);
  if (!(k.tmax > T_CUT)) return 0.0;
  return 0.5 * KBETHE * ZA / k.beta2 *
         ((1.0 / T_CUT - 1.0 / k.tmax) - k.beta2 / k.tmax * log(k.tmax / T_CUT));
}

double orc_omega2(double E) {
  kin_t k = kinematics(E);
  double tup = k.tmax < T_CUT ? k.tmax : T_CUT;
  return 0.5 * KBETHE * ZA / k.beta2 * (tup - k.beta2 * tup * tup / (2.0 * k.tmax));
}

/* Highland projected-angle variance for mass path L (g/cm^2) at energy E. */
double orc_highland_theta2(double E, double L) {
  if (!(L > 0.0)) return 0.0;
  kin_t k = kinematics(E);
  double x = L / X0W;
  double c = 1.0 + 0.038 * log(x / k.beta2);
  double a = 13.6 / k.pbc;
  return a * a * x * c * c;
}

/* ---------------------------------------------------------------------- */
/* tables                                                                  */
/* ---------------------------------------------------------------------- */
static const double GL_X[4] = {0.1834346424956498, 0.5255324099163290, 0.7966664774136267,
                               0.9602898564975363};
static const double GL_W[4] = {0.3626837833783620, 0.3137066458778873, 0.2223810344533745,
                               0.1012285362903763};

void orc_build_tables(orc_tables *t) {
  t->lnE0 = log(E_LO);
  t->dlnE = (log(E_HI) - log(E_LO)) / (double)(NTAB - 1);
  for (int i = 0; i < NTAB; ++i) {
    t->e[i] = exp(t->lnE0 + t->dlnE * i);
    t->mu_delta[i] = orc_mu_delta(t->e[i]);
    t->omega2[i] = orc_omega2(t->e[i]);
  }
  /* R(E_i) = integral from E_LO to E_i of dE / L(E), in u = ln E:
   * integrand E / L(E), 8-point Gauss-Legendre on each interval */
  t->R[0] = 0.0;
  for (int i = 0; i + 1 < NTAB; ++i) {
    double ua = t->lnE0 + t->dlnE * i, ub = t->lnE0 + t->dlnE * (i + 1);
    double mid = 0.5 * (ua + ub), half = 0.5 * (ub - ua), acc = 0.0;
    for (int q = 0; q < 4; ++q) {
      double e1 = exp(mid - half * GL_X[q]), e2 = exp(mid + half * GL_X[q]);
      acc += GL_W[q] * (e1 / orc_stopping_restricted(e1) + e2 / orc_stopping_restricted(e2));
    }
    t->R[i + 1] = t->R[i] + half * acc;
  }
}

static orc_tables G_T;
static pthread_once_t G_T_once = PTHREAD_ONCE_INIT;
static void init_tables(void) { orc_build_tables(&G_T); }
static const orc_tables *tables(void) {
  pthread_once(&G_T_once, init_tables);
  return &G_T;
}

/* every tabulated quantity is linear in ln E between nodes */
static double interp_t(const orc_tables *t, const double *tab, double E) {
  double x = (log(E) - t->lnE0) / t->dlnE;
  int i = (int)floor(x);
  if (i < 0) i = 0;
  if (i > NTAB - 2) i = NTAB - 2;
  double f = x - (double)i;
  return tab[i] + f * (tab[i + 1] - tab[i]);
}

/* exact inverse of the piecewise-linear (in ln E) range table */
static double rinv_t(const orc_tables *t, double R) {
  if (!(R > 0.0)) return E_LO;
  int lo = 0, hi = NTAB - 1;
  if (R >= t->R[NTAB - 1]) {
    lo = NTAB - 2;
  } else {
    while (hi - lo > 1) { /* invariant: R[lo] <= R < R[hi] */
      int mid = (lo + hi) / 2;
      if (t->R[mid] <= R) lo = mid; else hi = mid;
    }
  }
  double f = (R - t->R[lo]) / (t->R[lo + 1] - t->R[lo]);
  return exp(t->lnE0 + t->dlnE * ((double)lo + f));
}

double orc_interp(const double *tab, double E) { return interp_t(tables(), tab, E); }
double orc_range(double E) { return interp_t(tables(), tables()->R, E); }
double orc_range_inverse(double R) { return rinv_t(tables(), R); }

/* ---------------------------------------------------------------------- */
/* materials: piecewise-linear calibration at the clamped integer HU       */
/* ---------------------------------------------------------------------- */
static double calib_eval(const double *xh, const double *y, int n, double hu) {
  if (hu <= xh[0]) return y[0];
  if (hu >= xh[n - 1]) return y[n - 1];
  int i = 0;
  while (hu >= xh[i + 1]) ++i; /* xh[i] <= hu < xh[i+1] */
  return y[i] + (y[i + 1] - y[i]) * (hu - xh[i]) / (xh[i + 1] - xh[i]);
}

static void material(const orc_phase *ph, int16_t hu, double *rho, double *rsp) {
  int h = hu;
  if (h < HU_MIN) h = HU_MIN;
  if (h > HU_MAX) h = HU_MAX;
  *rho = calib_eval(ph->calib_hu, ph->calib_rho, ph->n_nodes, (double)h);
  *rsp = calib_eval(ph->calib_hu, ph->calib_rsp, ph->n_nodes, (double)h);
}

/* ---------------------------------------------------------------------- */
/* transport of one history                                                */
/* ---------------------------------------------------------------------- */
static inline int64_t Qe(double E) { return (int64_t)llrint(E * Q_SCALE); }

/* a / b with "zero coefficient => infinite distance" */
static inline double dist(double a, double b) { return b > 0.0 ? a / b : HUGE_VAL; }

typedef struct {
  const orc_phase *ph;
  const orc_field *fields;
  const orc_spot *spots;
  const orc_tables *T;
  uint32_t key[2];
  uint32_t flags;
  double d[3], ext[3];
  int n[3];
} hctx;

typedef struct {
  u128 incident, deposited, escaped, nuclear, cutoff;
  uint64_t histories, steps, delta_events, nuclear_events, escapes, misses;
} acc_t;

static void hctx_init(hctx *c, const orc_phase *ph, const orc_field *fields, const orc_spot *spots,
                      uint64_t seed, uint32_t request_id, uint32_t flags) {
  c->ph = ph;
  c->fields = fields;
  c->spots = spots;
  c->T = tables();
  c->key[0] = (uint32_t)(seed & 0xffffffffu);
  c->key[1] = request_id;
  c->flags = flags;
  c->n[0] = ph->nx; c->n[1] = ph->ny; c->n[2] = ph->nz;
  for (int k = 0; k < 3; ++k) {
    c->d[k] = ph->spacing_mm[k] * 0.1;
    c->ext[k] = c->n[k] * c->d[k];
  }
}

static void normalize3(double v[3]) {
  double n = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  v[0] /= n; v[1] /= n; v[2] /= n;
}

/* rotate unit vector w by polar angle theta and azimuth phi */
static void rotate(double w[3], double theta, double phi) {
  double ct = cos(theta), st = sin(theta), cp = cos(phi), sp = sin(phi);
  double a = w[0], b = w[1], c = w[2];
  double den2 = a * a + b * b;
  double na, nb, nc;
  if (den2 < 1e-20) {
    na = st * cp;
    nb = st * sp;
    nc = (c >= 0.0 ? 1.0 : -1.0) * ct;
  } else {
    double den = sqrt(den2);
    na = a * ct + st * (a * c * cp - b * sp) / den;
    nb = b * ct + st * (b * c * cp + a * sp) / den;
    nc = c * ct - st * cp * den;
  }
  double nn = sqrt(na * na + nb * nb + nc * nc);
  w[0] = na / nn; w[1] = nb / nn; w[2] = nc / nn;
}

static void trace_put(orc_trace_rec *rec, int32_t max_rec, int32_t *nrec, int cause, int64_t v,
                      int fate, uint32_t block, double s, double E, const double r[3],
                      const double w[3], double nd, double nn, double la, int64_t dep, double td,
                      double margin) {
  if (!rec || *nrec >= max_rec) { if (rec) ++*nrec; return; }
  orc_trace_rec *p = &rec[*nrec];
  p->cause = cause; p->voxel = (int32_t)v; p->fate = fate; p->block = block;
  p->s = s; p->E = E;
  for (int k = 0; k < 3; ++k) { p->r[k] = r[k]; p->w[k] = w[k]; }
  p->n_delta = nd; p->n_nuc = nn; p->l_acc = la; p->dep = dep; p->t_delta = td;
  p->margin = margin;
  ++*nrec;
}

/* Decision margins (traces only): the relative gap |a - b| / max(|a|, |b|)
 * of a comparison of a with b, folded into *m by min.  Infinite operands
 * (a zero coefficient) decide nothing. */
static inline void gap(double *m, double a, double b) {
  if (!m || isinf(a) || isinf(b)) return;
  double x = fabs(a) > fabs(b) ? fabs(a) : fabs(b);
  double g = x > 0.0 ? fabs(a - b) / x : 0.0;
  if (g < *m) *m = g;
}

/* the gap of the smallest of n values to the next smallest */
static void gap_min2(double *m, const double *x, int n) {
  if (!m) return;
  double a = HUGE_VAL, b = HUGE_VAL;
  for (int i = 0; i < n; ++i) {
    if (x[i] < a) { b = a; a = x[i]; }
    else if (x[i] < b) b = x[i];
  }
  gap(m, a, b);
}

/* Hard delta-ray energy: T from the 1/T^2 part of the free-electron spectrum
 * on [T_cut, Tmax] by inversion, accepted with probability 1 - beta^2 T/Tmax.
 * Each block gives two trials, (u0,u1) and (u2,u3). */
static double sample_delta(const uint32_t key[2], uint32_t *block, uint32_t h, uint32_t s,
                           kin_t k, double *m) {
  for (;;) {
    double q[4];
    draw4(key, (*block)++, h, s, q);
    double t1 = 1.0 / (1.0 / T_CUT - q[0] * (1.0 / T_CUT - 1.0 / k.tmax));
    gap(m, q[1], 1.0 - k.beta2 * t1 / k.tmax);
    if (q[1] < 1.0 - k.beta2 * t1 / k.tmax) return t1;
    double t2 = 1.0 / (1.0 / T_CUT - q[2] * (1.0 / T_CUT - 1.0 / k.tmax));
    gap(m, q[3], 1.0 - k.beta2 * t2 / k.tmax);
    if (q[3] < 1.0 - k.beta2 * t2 / k.tmax) return t2;
  }
}

static void transport(const hctx *c, int64_t spot, uint32_t h, int64_t *tally, acc_t *acc,
                      orc_trace_rec *rec, int32_t max_rec, int32_t *nrec) {
  const orc_spot *sp = &c->spots[spot];
  const orc_field *f = &c->fields[sp->field];
  const orc_phase *ph = c->ph;
  const orc_tables *T = c->T;
  const uint32_t flags = c->flags;
  const uint32_t s32 = (uint32_t)spot;
  double w[3], bu[3], bv[3];
  for (int k = 0; k < 3; ++k) { w[k] = f->direction[k]; bu[k] = f->bev_u[k]; }
  normalize3(w);
  normalize3(bu);
  bv[0] = w[1] * bu[2] - w[2] * bu[1];
  bv[1] = w[2] * bu[0] - w[0] * bu[2];
  bv[2] = w[0] * bu[1] - w[1] * bu[0];

  /* source: block 0 -> lateral Gaussian pair (Box-Muller), nuclear and delta
   * interaction lengths in mean free paths */
  double u[4];
  draw4(c->key, 0u, h, s32, u);
  double rad = sqrt(-2.0 * log(u[0]));
  double gx = rad * cos(TWO_PI * u[1]), gy = rad * sin(TWO_PI * u[1]);
  double n_nuc = -log(u[2]), n_delta = -log(u[3]);
  double E = sp->energy_MeV;
  acc->histories++;
  acc->incident += (u128)Qe(E);
  double a = 0.1 * sp->x_mm + 0.1 * sp->sigma_mm * gx;
  double b = 0.1 * sp->y_mm + 0.1 * sp->sigma_mm * gy;
  double p[3], r[3];
  for (int k = 0; k < 3; ++k)
    p[k] = 0.1 * (f->isocentre_mm[k] - ph->origin_mm[k]) + a * bu[k] + b * bv[k];

  /* decision margin of the step being traced (NULL: not tracing) */
  double mg_val = HUGE_VAL, *mg = rec ? &mg_val : NULL;
  /* entry into the grid box [0, ext) along the line p + t w (slab method) */
  double tn = -HUGE_VAL, tf = HUGE_VAL;
  double t_lo[3] = {-HUGE_VAL, -HUGE_VAL, -HUGE_VAL};
  int an = -1, missed = 0;
  for (int k = 0; k < 3; ++k) {
    if (w[k] != 0.0) {
      double t1 = (0.0 - p[k]) / w[k], t2 = (c->ext[k] - p[k]) / w[k];
      double lo = t1 < t2 ? t1 : t2, hi = t1 < t2 ? t2 : t1;
      t_lo[k] = lo;
      if (lo > tn) { tn = lo; an = k; }
      if (hi < tf) tf = hi;
    } else if (p[k] < 0.0 || p[k] >= c->ext[k]) {
      missed = 1;
    }
  }
  if (mg) { /* which face is entered, and whether the box is hit at all */
    double neg[3] = {-t_lo[0], -t_lo[1], -t_lo[2]};
    gap_min2(mg, neg, 3);
    gap(mg, tn, tf);
  }
  if (an < 0 || !(tn < tf)) missed = 1;
  if (missed) {
    acc->escaped += (u128)Qe(E);
    acc->misses++;
    trace_put(rec, max_rec, nrec, -1, -1, ORC_FATE_MISSED, 1u, 0.0, E, p, w, n_delta, n_nuc, 0.0, 0, 0.0,
              HUGE_VAL);
    return;
  }
  int idx[3];
  for (int k = 0; k < 3; ++k) r[k] = p[k] + tn * w[k];
  r[an] = w[an] > 0.0 ? 0.0 : c->ext[an];
  for (int k = 0; k < 3; ++k) {
    if (k == an) {
      idx[k] = w[k] > 0.0 ? 0 : c->n[k] - 1;
    } else {
      double q = r[k] / c->d[k];
      int i = (int)floor(q);
      gap(mg, q, floor(q + 0.5)); /* a coordinate on a voxel face */
      if (i < 0) i = 0;
      if (i > c->n[k] - 1) i = c->n[k] - 1;
      idx[k] = i;
    }
  }
  int64_t v = (int64_t)idx[0] + (int64_t)c->n[0] * ((int64_t)idx[1] + (int64_t)c->n[1] * idx[2]);
  uint32_t block = 1u;
  double l_acc = 0.0;
  trace_put(rec, max_rec, nrec, -1, v, ORC_FATE_ALIVE, block, 0.0, E, r, w, n_delta, n_nuc, l_acc, 0, 0.0,
            mg_val);

  int fate = ORC_FATE_ALIVE;
  uint64_t steps = 0;
  while (fate == ORC_FATE_ALIVE) {
    if (++steps > MAX_STEPS) { /* safety valve; never reached by valid input */
      acc->escaped += (u128)Qe(E);
      acc->escapes++;
      break;
    }
    mg_val = HUGE_VAL;
    /* 1. material of the current voxel */
    double rho, rsp;
    material(ph, ph->hu[v], &rho, &rsp);
    int vac = ph->mask != NULL && ph->mask[v] == 0;

    /* 2. distance to the voxel boundary; lowest axis wins ties */
    double dgeo = HUGE_VAL;
    int ax = -1;
    double t_ax[3] = {HUGE_VAL, HUGE_VAL, HUGE_VAL};
    for (int k = 0; k < 3; ++k) {
      double t;
      if (w[k] > 0.0) t = ((double)(idx[k] + 1) * c->d[k] - r[k]) / w[k];
      else if (w[k] < 0.0) t = ((double)idx[k] * c->d[k] - r[k]) / w[k];
      else continue;
      if (t < 0.0) t = 0.0;
      t_ax[k] = t;
      if (t < dgeo) { dgeo = t; ax = k; }
    }
    gap_min2(mg, t_ax, 3); /* which face is reached first */

    /* 3-4. physics limits and the step; priority on ties:
     * stop > geo > delta > nuclear > phys */
    double s = dgeo, R = 0.0, mud = 0.0, om2 = 0.0, mun = 0.0;
    int cause = ORC_CAUSE_GEO;
    if (!vac) {
      R = interp_t(T, T->R, E);
      mud = (flags & ORC_NO_DELTA) ? 0.0 : interp_t(T, T->mu_delta, E);
      om2 = interp_t(T, T->omega2, E);
      mun = (!(flags & ORC_NO_NUCLEAR) && E >= E_N) ? MU_N : 0.0;
      double s_stop = (flags & ORC_FROZEN) ? HUGE_VAL : dist(R, rsp);
      double s_phys = dist(fmax(EPS_R * R, S_FLOOR), rsp);
      double d_del = dist(n_delta, mud * rsp);
      double d_nuc = dist(n_nuc, mun * rho);
      if (d_del < 0.0) d_del = 0.0; /* rounding can leave a counter a hair below 0 */
      if (d_nuc < 0.0) d_nuc = 0.0;
      if (mg) { /* which limit is the shortest; the nuclear switch at E_N */
        double cand[5] = {s_stop, dgeo, d_del, d_nuc, s_phys};
        gap_min2(mg, cand, 5);
        if (!(flags & ORC_NO_NUCLEAR)) gap(mg, E, E_N);
      }
      s = s_stop;
      cause = ORC_CAUSE_STOP;
      if (dgeo < s) { s = dgeo; cause = ORC_CAUSE_GEO; }
      if (d_del < s) { s = d_del; cause = ORC_CAUSE_DELTA; }
      if (d_nuc < s) { s = d_nuc; cause = ORC_CAUSE_NUCLEAR; }
      if (s_phys < s) { s = s_phys; cause = ORC_CAUSE_PHYS; }
    }
    /* one fresh block per step: u0,u1 straggling; u2,u3 scattering */
    draw4(c->key, block++, h, s32, u);

    /* 5. move; a boundary crossing lands exactly on the face */
    int ax_pos = ax >= 0 && w[ax] > 0.0;
    for (int k = 0; k < 3; ++k) r[k] += s * w[k];
    if (cause == ORC_CAUSE_GEO)
      r[ax] = ax_pos ? (double)(idx[ax] + 1) * c->d[ax] : (double)idx[ax] * c->d[ax];

    const double E_pre = E;
    int64_t dep = 0;
    double t_delta = 0.0;
    if (!vac) {
      /* 6. continuous loss with Gaussian soft straggling */
      if (!(flags & ORC_FROZEN)) {
        if (cause == ORC_CAUSE_STOP) {
          fate = ORC_FATE_STOPPED;
        } else {
          double sw = rsp * s;
          double g = (flags & ORC_NO_STRAGGLING) ? 0.0 : sqrt(-2.0 * log(u[0])) * cos(TWO_PI * u[1]);
          double dE = (E - rinv_t(T, R - sw)) + sqrt(om2 * sw) * g;
          gap(mg, dE + E, E); /* the clamps of the loss to [0, E], and the cutoff */
          gap(mg, dE, E);
          if (dE < 0.0) dE = 0.0;
          if (dE > E) dE = E;
          double En = E - dE;
          gap(mg, En, E_LO);
          if (En <= E_LO) fate = ORC_FATE_STOPPED;
          else E = En;
        }
      }
      /* 7. interaction-length bookkeeping with pre-step coefficients */
      n_delta -= mud * rsp * s;
      n_nuc -= mun * rho * s;
      if (cause == ORC_CAUSE_DELTA) n_delta = 0.0;
      if (cause == ORC_CAUSE_NUCLEAR) n_nuc = 0.0;
      /* 8. telescoping Highland scattering at the pre-step energy */
      double l_new = l_acc + rho * s;
      double th2 = orc_highland_theta2(E_pre, l_new) - orc_highland_theta2(E_pre, l_acc);
      if (th2 < 0.0) th2 = 0.0;
      l_acc = l_new;
      if (fate == ORC_FATE_ALIVE && !(flags & ORC_NO_MCS) && th2 > 0.0) {
        double theta = sqrt(th2) * sqrt(-2.0 * log(u[2]));
        rotate(w, theta, TWO_PI * u[3]);
      }
      /* 9. tally by telescoping the fixed-point energy */
      if (fate == ORC_FATE_STOPPED) {
        dep = Qe(E_pre);
        acc->cutoff += (u128)Qe(E_pre);
      } else {
        dep = Qe(E_pre) - Qe(E);
      }
      /* 10. events at the step end */
      if (fate == ORC_FATE_ALIVE && cause == ORC_CAUSE_DELTA) {
        kin_t k = kinematics(E);
        gap(mg, k.tmax, T_CUT);
        if (k.tmax > T_CUT) {
          double T_d = sample_delta(c->key, &block, h, s32, k, mg);
          gap(mg, T_d, E - E_LO);
          if (T_d > E - E_LO) T_d = E - E_LO;
          t_delta = T_d;
          acc->delta_events++;
          if (!(flags & ORC_FROZEN)) {
            double En = E - T_d;
            dep += Qe(E) - Qe(En);
            E = En;
            gap(mg, E, E_LO);
            if (E <= E_LO) {
              dep += Qe(E);
              acc->cutoff += (u128)Qe(E);
              fate = ORC_FATE_STOPPED;
            }
          }
        }
        double q[4];
        draw4(c->key, block++, h, s32, q);
        n_delta = -log(q[0]);
      } else if (fate == ORC_FATE_ALIVE && cause == ORC_CAUSE_NUCLEAR) {
        acc->nuclear += (u128)Qe(E);
        acc->nuclear_events++;
        fate = ORC_FATE_NUCLEAR;
      }
      if (dep != 0 && tally) __atomic_fetch_add(&tally[v], dep, __ATOMIC_RELAXED);
      acc->deposited += (u128)dep;
    }
    acc->steps++;
    int64_t v_step = v;
    /* 11. voxel crossing */
    if (fate == ORC_FATE_ALIVE && cause == ORC_CAUSE_GEO) {
      idx[ax] += ax_pos ? 1 : -1;
      if (idx[ax] < 0 || idx[ax] >= c->n[ax]) {
        acc->escaped += (u128)Qe(E);
        acc->escapes++;
        fate = ORC_FATE_ESCAPED;
      } else {
        v = (int64_t)idx[0] + (int64_t)c->n[0] * ((int64_t)idx[1] + (int64_t)c->n[1] * idx[2]);
      }
    }
    double E_rec = (fate == ORC_FATE_STOPPED) ? 0.0 : E;
    trace_put(rec, max_rec, nrec, cause, v_step, fate, block, s, E_rec, r, w, n_delta, n_nuc, l_acc,
              dep, t_delta, mg_val);
  }
}

/* ---------------------------------------------------------------------- */
/* history split: largest remainder, ties to the lower spot index          */
/* ---------------------------------------------------------------------- */
typedef struct { double rem; int64_t idx; } rem_t;

static int rem_cmp(const void *pa, const void *pb) {
  const rem_t *a = (const rem_t *)pa, *b = (const rem_t *)pb;
  if (a->rem > b->rem) return -1;
  if (a->rem < b->rem) return 1;
  return a->idx < b->idx ? -1 : (a->idx > b->idx ? 1 : 0);
}

static int listed(int32_t phase, const int32_t *ids, int32_t n) {
  for (int32_t i = 0; i < n; ++i)
    if (ids[i] == phase) return i;
  return -1;
}

int orc_split_histories(const orc_spot *spots, int64_t n_spots, const int32_t *phase_ids,
                        int32_t n_req_phases, uint64_t n_hist, int64_t *per_spot) {
  double W = 0.0;
  int64_t m = 0;
  for (int64_t s = 0; s < n_spots; ++s) {
    per_spot[s] = 0;
    if (listed(spots[s].phase, phase_ids, n_req_phases) >= 0) { W += spots[s].weight; ++m; }
  }
  if (m == 0 || !(W > 0.0)) return -1;
  rem_t *r = (rem_t *)malloc(sizeof(rem_t) * (size_t)m);
  if (!r) return -2;
  uint64_t assigned = 0;
  int64_t j = 0;
  for (int64_t s = 0; s < n_spots; ++s) {
    if (listed(spots[s].phase, phase_ids, n_req_phases) < 0) continue;
    double q = (double)n_hist * spots[s].weight / W;
    double fl = floor(q);
    per_spot[s] = (int64_t)fl;
    assigned += (uint64_t)fl;
    r[j].rem = q - fl;
    r[j].idx = s;
    ++j;
  }
  qsort(r, (size_t)m, sizeof(rem_t), rem_cmp);
  uint64_t left = n_hist > assigned ? n_hist - assigned : 0;
  for (int64_t k = 0; k < m && left > 0; ++k, --left) per_spot[r[k].idx] += 1;
  free(r);
  return 0;
}

/* ---------------------------------------------------------------------- */
/* threaded run                                                            */
/* ---------------------------------------------------------------------- */
typedef struct {
  const orc_phase *phases;
  const orc_field *fields;
  const orc_spot *spots;
  const int32_t *slot_of_spot; /* tally slot (position in the request) or -1 */
  const int32_t *phase_ids;
  const int64_t *offset;       /* prefix sum of per-spot histories */
  const int64_t *count;
  int64_t n_spots;
  int64_t s_begin, s_end;       /* only spots s_begin <= s < s_end run */
  int64_t *const *tallies;
  uint64_t seed;
  uint32_t request_id, flags, h_begin, h_end, h_mod, h_rem;
  int64_t g_begin, g_end;       /* range of the flattened history list */
  acc_t acc;
} job_t;

static void *job_run(void *arg) {
  job_t *j = (job_t *)arg;
  memset(&j->acc, 0, sizeof(j->acc));
  /* first spot containing g_begin */
  int64_t lo = 0, hi = j->n_spots;
  while (hi - lo > 1) {
    int64_t mid = (lo + hi) / 2;
    if (j->offset[mid] <= j->g_begin) lo = mid; else hi = mid;
  }
  hctx c;
  int64_t cur_slot = -2;
  for (int64_t s = lo; s < j->n_spots; ++s) {
    int64_t a = j->offset[s], e = a + j->count[s];
    if (a >= j->g_end) break;
    if (j->count[s] == 0 || j->slot_of_spot[s] < 0 || s < j->s_begin || s >= j->s_end) continue;
    int32_t slot = j->slot_of_spot[s];
    if (slot != cur_slot) {
      hctx_init(&c, &j->phases[j->phase_ids[slot]], j->fields, j->spots, j->seed, j->request_id,
                j->flags);
      cur_slot = slot;
    }
    int64_t g0 = a > j->g_begin ? a : j->g_begin;
    int64_t g1 = e < j->g_end ? e : j->g_end;
    for (int64_t g = g0; g < g1; ++g) {
      uint32_t h = (uint32_t)(g - a);
      if (h < j->h_begin || h >= j->h_end || h % j->h_mod != j->h_rem) continue;
      transport(&c, s, h, j->tallies[slot], &j->acc, NULL, 0, NULL);
    }
  }
  return NULL;
}

static void put128(uint64_t out[2], u128 v) {
  out[0] = (uint64_t)v;
  out[1] = (uint64_t)(v >> 64);
}

static int run_common(const orc_phase *phases, int32_t n_phases, const orc_field *fields,
                      int32_t n_fields, const orc_spot *spots, int64_t n_spots,
                      const int32_t *phase_ids, int32_t n_req_phases, uint64_t seed,
                      uint32_t request_id, uint64_t n_hist, uint32_t flags, int32_t n_threads,
                      uint32_t h_begin, uint32_t h_end, uint32_t h_mod, uint32_t h_rem,
                      int64_t s_begin, int64_t s_end, int64_t *const *tallies, orc_balance *bal) {
  if (h_mod == 0 || h_rem >= h_mod) return -1;
  if (n_phases <= 0 || n_req_phases <= 0 || n_spots <= 0 || n_hist == 0) return -1;
  for (int32_t i = 0; i < n_req_phases; ++i)
    if (phase_ids[i] < 0 || phase_ids[i] >= n_phases) return -1;
  for (int64_t s = 0; s < n_spots; ++s)
    if (spots[s].field < 0 || spots[s].field >= n_fields) return -1;
  int64_t *count = (int64_t *)calloc((size_t)n_spots, sizeof(int64_t));
  int64_t *offset = (int64_t *)calloc((size_t)n_spots + 1, sizeof(int64_t));
  int32_t *slot = (int32_t *)malloc(sizeof(int32_t) * (size_t)n_spots);
  if (!count || !offset || !slot) { free(count); free(offset); free(slot); return -2; }
  int rc = orc_split_histories(spots, n_spots, phase_ids, n_req_phases, n_hist, count);
  if (rc) { free(count); free(offset); free(slot); return rc; }
  for (int64_t s = 0; s < n_spots; ++s) {
    offset[s + 1] = offset[s] + count[s];
    slot[s] = listed(spots[s].phase, phase_ids, n_req_phases);
  }
  int64_t total = offset[n_spots];
  if (n_threads < 1) n_threads = 1;
  job_t *jobs = (job_t *)calloc((size_t)n_threads, sizeof(job_t));
  pthread_t *th = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
  for (int32_t t = 0; t < n_threads; ++t) {
    job_t *j = &jobs[t];
    j->phases = phases; j->fields = fields; j->spots = spots; j->slot_of_spot = slot;
    j->phase_ids = phase_ids; j->offset = offset; j->count = count; j->n_spots = n_spots;
    j->tallies = tallies; j->seed = seed; j->request_id = request_id; j->flags = flags;
    j->h_begin = h_begin; j->h_end = h_end; j->h_mod = h_mod; j->h_rem = h_rem;
    j->s_begin = s_begin; j->s_end = s_end;
    j->g_begin = total * t / n_threads;
    j->g_end = total * (t + 1) / n_threads;
  }
  tables();
  for (int32_t t = 1; t < n_threads; ++t) pthread_create(&th[t], NULL, job_run, &jobs[t]);
  job_run(&jobs[0]);
  for (int32_t t = 1; t < n_threads; ++t) pthread_join(th[t], NULL);
  acc_t sum;
  memset(&sum, 0, sizeof(sum));
  for (int32_t t = 0; t < n_threads; ++t) {
    acc_t *a = &jobs[t].acc;
    sum.incident += a->incident; sum.deposited += a->deposited; sum.escaped += a->escaped;
    sum.nuclear += a->nuclear; sum.cutoff += a->cutoff; sum.histories += a->histories;
    sum.steps += a->steps; sum.delta_events += a->delta_events;
    sum.nuclear_events += a->nuclear_events; sum.escapes += a->escapes; sum.misses += a->misses;
  }
  if (bal) {
    put128(bal->incident, sum.incident); put128(bal->deposited, sum.deposited);
    put128(bal->escaped, sum.escaped); put128(bal->nuclear, sum.nuclear);
    put128(bal->cutoff, sum.cutoff);
    bal->histories = sum.histories; bal->steps = sum.steps; bal->delta_events = sum.delta_events;
    bal->nuclear_events = sum.nuclear_events; bal->escapes = sum.escapes; bal->misses = sum.misses;
  }
  free(jobs); free(th); free(count); free(offset); free(slot);
  return 0;
}

int orc_dose(const orc_phase *phases, int32_t n_phases, const orc_field *fields, int32_t n_fields,
             const orc_spot *spots, int64_t n_spots, const int32_t *phase_ids, int32_t n_req_phases,
             uint64_t seed, uint32_t request_id, uint64_t n_hist, uint32_t flags, int32_t n_threads,
             int64_t *const *tallies, double *const *dose, orc_balance *bal) {
  int rc = run_common(phases, n_phases, fields, n_fields, spots, n_spots, phase_ids, n_req_phases,
                      seed, request_id, n_hist, flags, n_threads, 0u, 0xffffffffu, 1u, 0u, 0, n_spots,
                      tallies, bal);
  if (rc) return rc;
  if (dose)
    for (int32_t i = 0; i < n_req_phases; ++i)
      if (dose[i]) orc_convert(&phases[phase_ids[i]], tallies[i], n_hist, dose[i], NULL);
  return 0;
}

int orc_dose_subset(const orc_phase *phases, int32_t n_phases, const orc_field *fields,
                    int32_t n_fields, const orc_spot *spots, int64_t n_spots,
                    const int32_t *phase_ids, int32_t n_req_phases, uint64_t seed,
                    uint32_t request_id, uint64_t n_hist, uint32_t flags, int32_t n_threads,
                    uint32_t h_begin, uint32_t h_end, uint32_t h_mod, uint32_t h_rem,
                    int64_t *const *tallies, orc_balance *bal) {
  return run_common(phases, n_phases, fields, n_fields, spots, n_spots, phase_ids, n_req_phases,
                    seed, request_id, n_hist, flags, n_threads, h_begin, h_end, h_mod, h_rem, 0,
                    n_spots, tallies, bal);
}

int orc_dose_spots_batch(const orc_phase *phases, int32_t n_phases, const orc_field *fields,
                         int32_t n_fields, const orc_spot *spots, int64_t n_spots,
                         const int32_t *phase_ids, int32_t n_req_phases, uint64_t seed,
                         uint32_t request_id, uint64_t n_hist, uint32_t flags, int32_t n_threads,
                         int64_t s_begin, int64_t s_end, uint32_t h_mod, uint32_t h_rem,
                         int64_t *const *tallies, orc_balance *bal) {
  if (s_begin < 0 || s_end > n_spots || s_begin > s_end) return -1;
  return run_common(phases, n_phases, fields, n_fields, spots, n_spots, phase_ids, n_req_phases,
                    seed, request_id, n_hist, flags, n_threads, 0u, 0xffffffffu, h_mod, h_rem,
                    s_begin, s_end, tallies, bal);
}

int orc_dose_spots(const orc_phase *phases, int32_t n_phases, const orc_field *fields,
                   int32_t n_fields, const orc_spot *spots, int64_t n_spots,
                   const int32_t *phase_ids, int32_t n_req_phases, uint64_t seed,
                   uint32_t request_id, uint64_t n_hist, uint32_t flags, int32_t n_threads,
                   int64_t s_begin, int64_t s_end, int64_t *const *tallies, orc_balance *bal) {
  return orc_dose_spots_batch(phases, n_phases, fields, n_fields, spots, n_spots, phase_ids,
                              n_req_phases, seed, request_id, n_hist, flags, n_threads, s_begin,
                              s_end, 1u, 0u, tallies, bal);
}

int orc_trace(const orc_phase *phase, const orc_field *fields, int32_t n_fields,
              const orc_spot *spots, int64_t n_spots, int64_t spot, uint32_t h, uint64_t seed,
              uint32_t request_id, uint32_t flags, orc_trace_rec *rec, int32_t max_rec) {
  if (spot < 0 || spot >= n_spots || spots[spot].field < 0 || spots[spot].field >= n_fields)
    return -1;
  hctx c;
  hctx_init(&c, phase, fields, spots, seed, request_id, flags);
  acc_t acc;
  memset(&acc, 0, sizeof(acc));
  int32_t n = 0;
  transport(&c, spot, h, NULL, &acc, rec, max_rec, &n);
  return n;
}

int orc_sample_delta(double E, uint32_t seed, uint32_t request_id, uint32_t h, uint32_t s,
                     int32_t n, double *T_out) {
  kin_t k = kinematics(E);
  if (!(k.tmax > T_CUT)) return -1;
  uint32_t key[2] = {seed, request_id};
  uint32_t block = 0;
  for (int32_t i = 0; i < n; ++i) T_out[i] = sample_delta(key, &block, h, s, k, NULL);
  return 0;
}

/* Eq. (4) of the paper read backwards: D = E_dep / (rho V), in Gy per history */
int orc_convert(const orc_phase *ph, const int64_t *tally, uint64_t n_hist, double *dose,
                double *density) {
  if (n_hist == 0) return -1;
  double V = (ph->spacing_mm[0] * 0.1) * (ph->spacing_mm[1] * 0.1) * (ph->spacing_mm[2] * 0.1);
  int64_t nv = (int64_t)ph->nx * ph->ny * ph->nz;
  for (int64_t v = 0; v < nv; ++v) {
    double rho, rsp;
    material(ph, ph->hu[v], &rho, &rsp);
    if (ph->mask && ph->mask[v] == 0) rho = 0.0;
    if (density) density[v] = rho;
    if (dose) {
      if (rho > 0.0) {
        double e_j = (double)tally[v] / Q_SCALE * MEV_TO_J;
        double m_kg = rho * V * 1e-3;
        dose[v] = e_j / m_kg / (double)n_hist;
      } else {
        dose[v] = 0.0;
      }
    }
  }
  return 0;
}
