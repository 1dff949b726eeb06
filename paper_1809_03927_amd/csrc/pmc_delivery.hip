// Beam-delivery simulation (Sec. 2.B, App. A): which part of each spot's MU
// is delivered in which breathing phase.  One lane walks the timeline of one
// (trial, field): breathing phases of N(mu, sigma) / N, synchrotron fills
// (layer switch, wait for the gate, discarded beam), spills and spot switches,
// refills on charge or extraction time, isolayered repainting.  Every random
// number is a Philox word keyed by (seed, trial) at counter (field, purpose,
// index, block); a Gaussian N(0, 1) is the Box-Muller transform of the first
// two words of one block, in FP64.  The walk itself is the same sequence of
// FP64 operations on every run, so the result is reproducible bit for bit.
#include <hip/hip_runtime.h>

#include "pmc_device.hpp"

namespace pmc {

namespace {

enum : uint32_t { kPStart = 0, kPSync = 1, kPBreath = 2, kPPeriod = 3 };
enum { kSwitch = 0, kSwitchPerMev, kDiscard, kRate, kRatePerMev, kSpotSwitch, kSpotSwitchPerMm, kCapacity,
       kExtractionMax };
constexpr long long kMaxAdvances = 1LL << 30;  // breathing phases per thread before giving up

// z = sqrt(-2 ln u_a) cos(2 pi u_b), u = (x + 1/2) 2^-32 of the words x, y of
// block 0: |z| <= sqrt(66 ln 2) = 6.77 (the smallest u is 2^-33).
__device__ double gauss(uint32_t k0, uint32_t k1, uint32_t field, uint32_t purpose, uint32_t index) {
  const uint4 x = philox(field, purpose, index, 0u, k0, k1);
  const double ua = ((double)x.x + 0.5) * 0x1p-32;
  const double ub = ((double)x.y + 0.5) * 0x1p-32;
  return sqrt(-2.0 * log(ua)) * cos(6.283185307179586 * ub);
}

__device__ __forceinline__ int draw_int(uint32_t k0, uint32_t k1, uint32_t field, uint32_t purpose, uint32_t n) {
  const uint4 x = philox(field, purpose, 0u, 0u, k0, k1);
  return (int)(((unsigned long long)x.x * n) >> 32);
}

// The breathing timeline of one (trial, field): occurrence k of a phase is
// phase (phi0 + k) mod N and lasts max(mu + sigma z_k, mu / 20) / N.
struct Breathing {
  uint32_t k0, k1, field;
  int n, phi0, gate_lo, gate_hi;
  double mu, sd;
  long long k, advances;
  double t0, t1;

  __device__ double length(long long kk) const {
    double p = mu + sd * gauss(k0, k1, field, kPBreath, (uint32_t)kk);
    if (p < mu / 20.0) p = mu / 20.0;
    return p / (double)n;
  }
  __device__ int phase(double t) {
    while (t >= t1 && advances < kMaxAdvances) {
      ++k;
      ++advances;
      t0 = t1;
      t1 = t0 + length(k);
    }
    return (int)((phi0 + k) % n);
  }
  __device__ bool open(int ph) const { return gate_lo < 0 || (gate_lo <= ph && ph <= gate_hi); }
  // the first time >= t at which the gate is open
  __device__ double wait_gate(double t) {
    int ph = phase(t);
    while (!open(ph) && advances < kMaxAdvances) {
      t = t1;
      ph = phase(t);
    }
    return t;
  }
};

// One 64-thread block per (trial, field).  Lane 0 walks the timeline; for
// every layer of at most layer_cap spots all lanes first stage its spots in
// LDS and zero per-(spot, phase) MU sums there, lane 0 adds each delivery
// into them (in delivery order, as a walk over global memory would), and all
// lanes then store the sums to the output.  Longer layers are walked over
// global memory (the output is zeroed by the caller).
__global__ void __launch_bounds__(64) delivery_sim(DeliveryLaunch a) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_i, s_j;
  const int n_ph = a.n_phases;
  DeliverySpot *lsp = reinterpret_cast<DeliverySpot *>(smem);
  double *lacc = reinterpret_cast<double *>(smem + sizeof(DeliverySpot) * (size_t)a.layer_cap);
  const int trial = (int)(blockIdx.x / (unsigned)a.n_fields), field = (int)(blockIdx.x % (unsigned)a.n_fields);
  const int s0 = a.fstart[field], s1 = a.fstart[field + 1];
  const bool lead = threadIdx.x == 0;
  const uint32_t k0 = a.seed, k1 = (uint32_t)trial;
  const long long out0 = (long long)trial * a.n_spots;
  // lane 0's timeline state
  double par[kSyncParams];
  Breathing br;
  double t = 0.0;
  int fills = 0;
  int i = s0;
  if (lead) {
    for (int p = 0; p < kSyncParams; ++p) {
      const double v = a.central[p] + a.sd[p] * gauss(k0, k1, (uint32_t)field, kPSync, (uint32_t)p);
      par[p] = v > 0.0 ? v : 0.0;
    }
    br.k0 = k0;
    br.k1 = k1;
    br.field = (uint32_t)field;
    br.n = n_ph;
    br.phi0 = a.start_phase >= 0 ? a.start_phase : draw_int(k0, k1, (uint32_t)field, kPStart, (uint32_t)n_ph);
    br.gate_lo = a.gate_lo;
    br.gate_hi = a.gate_hi;
    br.mu = (a.period_min > 0 && a.period_min <= a.period_max)
                ? (double)(a.period_min + draw_int(k0, k1, (uint32_t)field, kPPeriod,
                                                   (uint32_t)(a.period_max - a.period_min + 1)))
                : a.period_s;
    br.sd = a.period_sd_s;
    br.k = 0;
    br.advances = 0;
    br.t0 = 0.0;
    br.t1 = br.length(0);
  }
  const bool gated = a.gate_lo >= 0;
  for (;;) {
    if (lead) {
      // the next layer: consecutive spots of one energy
      int j = i;
      if (i < s1) {
        const double e = a.spots[i].e;
        j = i + 1;
        while (j < s1 && a.spots[j].e == e) ++j;
      }
      s_i = i;
      s_j = j;
    }
    __syncthreads();
    const int li = s_i, lj = s_j;
    if (li >= s1) break;
    const int n_l = lj - li;
    const bool staged = n_l <= a.layer_cap;
    if (staged) {
      for (int k = threadIdx.x; k < n_l; k += 64) lsp[k] = a.spots[li + k];
      for (int k = threadIdx.x; k < n_l * n_ph; k += 64) lacc[k] = 0.0;
    }
    __syncthreads();
    if (lead) {
      const DeliverySpot *sp_l = staged ? lsp : a.spots + li;
      const double e = sp_l[0].e;
      const double sw = par[kSwitch] + par[kSwitchPerMev] * (e - 70.0);
      const double rate = par[kRate] + par[kRatePerMev] * (e - 70.0);
      t = t + sw;
      t = br.wait_gate(t) + par[kDiscard];
      double t_ext = t;
      double q = par[kCapacity];
      ++fills;
      bool fresh = true, have_prev = false;
      double px = 0.0, py = 0.0;
      for (int r = 0;; ++r) {
        bool any = false;
        for (int s = 0; s < n_l; ++s) {
          const DeliverySpot sp = sp_l[s];
          double m;
          if (a.max_mu > 0.0) {
            m = sp.mu - (double)r * a.max_mu;
            if (m > a.max_mu) m = a.max_mu;
          } else {
            m = r == 0 ? sp.mu : 0.0;
          }
          if (m <= 0.0) continue;
          any = true;
          if (have_prev) {
            const double dx = fabs(sp.x - px), dy = fabs(sp.y - py);
            t = t + (par[kSpotSwitch] + par[kSpotSwitchPerMm] * (dx > dy ? dx : dy));
          }
          const double spill = m / rate;
          if (!fresh && (m > q || (t - t_ext) + spill > par[kExtractionMax])) {
            t = t + sw;
            t = br.wait_gate(t) + par[kDiscard];
            t_ext = t;
            q = par[kCapacity];
            ++fills;
          }
          if (gated && !br.open(br.phase(t))) t = br.wait_gate(t) + par[kDiscard];
          const int ph = br.phase(t);
          double *cell = staged ? lacc + (long long)s * n_ph + ph
                                : a.mu + (out0 + a.index[li + s]) * n_ph + ph;
          *cell = *cell + m;
          t = t + spill;
          q = q - m;
          fresh = false;
          have_prev = true;
          px = sp.x;
          py = sp.y;
        }
        if (!any || br.advances >= kMaxAdvances) break;
      }
      // past the cap the timeline is abandoned (the caller reports an error)
      i = br.advances >= kMaxAdvances ? s1 : lj;
    }
    __syncthreads();
    if (staged) {
      for (int k = threadIdx.x; k < n_l * n_ph; k += 64) {
        const int s = k / n_ph, ph = k - s * n_ph;
        a.mu[(out0 + a.index[li + s]) * n_ph + ph] = lacc[k];
      }
    }
    __syncthreads();
  }
  if (lead) {
    if (br.advances >= kMaxAdvances) a.status[0] = 1;
    a.time[blockIdx.x] = t;
    a.fills[blockIdx.x] = fills;
  }
}

}  // namespace

hipError_t launch_delivery(const DeliveryLaunch &a, hipStream_t st) {
  const long long n = (long long)a.n_trials * a.n_fields;
  const size_t lds = (sizeof(DeliverySpot) + sizeof(double) * (size_t)a.n_phases) * (size_t)a.layer_cap;
  if (n < 1 || n > (1LL << 31) - 1 || lds > 65536) return hipErrorInvalidValue;
  hipLaunchKernelGGL(delivery_sim, dim3((unsigned)n), dim3(64), lds, st, a);
  return hipGetLastError();
}

}  // namespace pmc
