// Physics tables of the transport model, built once per context on the host
// in double precision and uploaded in the working precision.
//
// Water, per unit mass thickness (PDG review "Passage of particles through
// matter"; Bethe theory without shell or density corrections, I = 75 eV):
//   restricted stopping power  L(E)  (energy transfers below T_cut),
//   hard-delta coefficient     mu(E) (integral of the free-electron spectrum
//                                     of a spin-1/2 projectile above T_cut),
//   soft straggling variance   w2(E) (second moment below min(T_cut, Tmax)),
//   restricted CSDA range      R(E) = integral_{E_lo}^{E} dE' / L(E').
// Nodes are uniform in ln E from 1 to 300 MeV; R uses 8-point Gauss-Legendre
// in ln E on every interval.
#include <cmath>

#include "pmc_internal.hpp"

namespace pmc {
namespace {

constexpr double kElectron = 0.51099895;   // MeV
constexpr double kProton = 938.27208816;   // MeV
constexpr double kBethe = 0.307075;        // MeV cm^2 / mol
constexpr double kZoverA = 0.555087;       // mol / g, water
constexpr double kIexc = 75.0e-6;          // MeV
constexpr double kTcutMeV = 0.1;
constexpr double kEmin = 1.0, kEmax = 300.0;

struct Kinematics {
  double beta2, bg2, tmax;
  explicit Kinematics(double T) {
    const double gam = 1.0 + T / kProton;
    bg2 = gam * gam - 1.0;
    beta2 = 1.0 - 1.0 / (gam * gam);
    const double ratio = kElectron / kProton;
    tmax = 2.0 * kElectron * bg2 / (1.0 + 2.0 * gam * ratio + ratio * ratio);
  }
};

double restricted_stopping(double T) {
  const Kinematics k(T);
  const double tup = std::fmin(kTcutMeV, k.tmax);
  const double pre = kBethe * kZoverA / k.beta2;
  return pre * (0.5 * std::log(2.0 * kElectron * k.bg2 * tup / (kIexc * kIexc)) -
                0.5 * k.beta2 * (1.0 + tup / k.tmax));
}

double hard_delta_coefficient(double T) {
  const Kinematics k(T);
  if (!(k.tmax > kTcutMeV)) return 0.0;
  const double pre = 0.5 * kBethe * kZoverA / k.beta2;
  return pre * ((1.0 / kTcutMeV - 1.0 / k.tmax) - k.beta2 / k.tmax * std::log(k.tmax / kTcutMeV));
}

double soft_variance(double T) {
  const Kinematics k(T);
  const double tup = std::fmin(kTcutMeV, k.tmax);
  const double pre = 0.5 * kBethe * kZoverA / k.beta2;
  return pre * (tup - k.beta2 * tup * tup / (2.0 * k.tmax));
}

// 8-point Gauss-Legendre abscissae and weights on [-1, 1] (symmetric pairs)
constexpr double kGaussX[4] = {0.1834346424956498, 0.5255324099163290, 0.7966664774136267,
                               0.9602898564975363};
constexpr double kGaussW[4] = {0.3626837833783620, 0.3137066458778873, 0.2223810344533745,
                               0.1012285362903763};

}  // namespace

void build_tables(Tables *t) {
  const double u0 = std::log(kEmin);
  const double du = (std::log(kEmax) - std::log(kEmin)) / (kTableNodes - 1);
  for (int i = 0; i < kTableNodes; ++i) {
    t->lnE[i] = u0 + du * i;
    const double E = std::exp(t->lnE[i]);
    t->mu_delta[i] = hard_delta_coefficient(E);
    t->omega2[i] = soft_variance(E);
  }
  t->range[0] = 0.0;
  for (int i = 1; i < kTableNodes; ++i) {
    const double a = t->lnE[i - 1], b = t->lnE[i];
    const double c = 0.5 * (a + b), h = 0.5 * (b - a);
    double sum = 0.0;
    for (int q = 0; q < 4; ++q) {
      for (int sgn = -1; sgn <= 1; sgn += 2) {
        const double E = std::exp(c + sgn * h * kGaussX[q]);
        sum += kGaussW[q] * E / restricted_stopping(E);
      }
    }
    t->range[i] = t->range[i - 1] + h * sum;
  }
  t->l2e0 = std::log2(kEmin);
  t->dl2 = (std::log2(kEmax) - std::log2(kEmin)) / (kTableNodes - 1);
}

}  // namespace pmc
