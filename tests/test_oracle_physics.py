"""Pins of the oracle's physics functions and tables against external facts.

Each check compares the oracle with something other than itself: tabulated
textbook data (NIST PSTAR), numerical integration of the differential
delta-ray spectrum from the PDG review (a different expression from the
oracle's closed forms), the relativistic Bohr straggling formula, and an
independent adaptive quadrature of the range integral.
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import integrate

HERE = os.path.dirname(os.path.abspath(__file__))

# constants written out independently of the oracle (PDG / CODATA)
ME = 0.51099895
MP = 938.27208816
K = 0.307075
ZA = 0.555087
TCUT = 0.1


def pstar():
    rows = []
    with open(os.path.join(HERE, "golden", "pstar_water.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([float(x) for x in line.split()])
    return np.array(rows)


def kin(T):
    """beta^2 and Tmax from momentum and total energy (a different route)."""
    Etot = T + MP
    pc = math.sqrt(T * T + 2 * T * MP)
    beta2 = (pc / Etot) ** 2
    gamma = Etot / MP
    tmax = 2 * ME * beta2 * gamma ** 2 / (1 + 2 * gamma * ME / MP + (ME / MP) ** 2)
    return beta2, tmax


def spectrum(T, beta2, tmax):
    """PDG free-electron spectrum per unit mass thickness: d mu / dT."""
    return 0.5 * K * ZA / beta2 * (1.0 - beta2 * T / tmax) / (T * T)


@pytest.mark.parametrize("row", range(6))
def test_stopping_power_vs_pstar(orc, row):
    E, S_ref, _ = pstar()[row]
    S = orc.f64("orc_stopping_unrestricted", E)
    # no shell or density corrections in the model: 2 % at 10-20 MeV, 0.5 % above
    tol = 0.02 if E < 50 else 0.005
    assert abs(S / S_ref - 1) < tol, (E, S, S_ref)


@pytest.mark.parametrize("row", range(1, 6))
def test_csda_range_vs_pstar(orc, row):
    E, _, R_ref = pstar()[row]
    # model CSDA range: PSTAR's range at the 1 MeV floor plus the integral of 1/S above
    R1 = 0.002458  # PSTAR CSDA range at 1 MeV, g/cm^2
    Rm = R1 + integrate.quad(lambda e: 1.0 / orc.f64("orc_stopping_unrestricted", e), 1.0, E,
                             limit=400, epsrel=1e-10)[0]
    assert abs(Rm / R_ref - 1) < 0.01, (E, Rm, R_ref)


@pytest.mark.parametrize("E", [46.0, 60.0, 100.0, 150.0, 200.0, 250.0, 299.0])
def test_delta_coefficients_vs_spectrum(orc, E):
    """mu_delta, S - L and omega2 against numerical integrals of the spectrum."""
    beta2, tmax = kin(E)
    assert tmax > TCUT
    mu = integrate.quad(lambda t: spectrum(t, beta2, tmax), TCUT, tmax, epsrel=1e-12)[0]
    hard = integrate.quad(lambda t: t * spectrum(t, beta2, tmax), TCUT, tmax, epsrel=1e-12)[0]
    soft2 = integrate.quad(lambda t: t * t * spectrum(t, beta2, tmax), 0.0, TCUT, epsrel=1e-12)[0]
    assert orc.f64("orc_mu_delta", E) == pytest.approx(mu, rel=1e-9)
    S = orc.f64("orc_stopping_unrestricted", E)
    L = orc.f64("orc_stopping_restricted", E)
    assert S - L == pytest.approx(hard, rel=1e-9)
    assert orc.f64("orc_omega2", E) == pytest.approx(soft2, rel=1e-9)


@pytest.mark.parametrize("E", [2.0, 10.0, 30.0, 44.0])
def test_omega2_is_relativistic_bohr_below_threshold(orc, E):
    """With Tmax < T_cut the whole spectrum is soft and omega^2 is Bohr's
    variance K (Z/A) m_e c^2 (1 - beta^2/2) / (1 - beta^2) (up to the
    projectile-mass term in Tmax, < 0.2 %)."""
    beta2, tmax = kin(E)
    assert tmax < TCUT
    bohr = K * ZA * ME * (1 - beta2 / 2) / (1 - beta2)
    assert orc.f64("orc_omega2", E) == pytest.approx(bohr, rel=2e-3)
    assert orc.f64("orc_mu_delta", E) == 0.0
    assert orc.f64("orc_stopping_unrestricted", E) == pytest.approx(
        orc.f64("orc_stopping_restricted", E), rel=1e-12)


def test_range_table_is_the_integral_of_1_over_L(orc):
    t = orc.tables()
    e = np.array(t.e)
    R = np.array(t.R)
    assert R[0] == 0.0 and e[0] == pytest.approx(1.0) and e[-1] == pytest.approx(300.0)
    assert np.all(np.diff(R) > 0)
    for i in (1, 10, 100, 400, 700, 1023):
        ref = integrate.quad(lambda x: 1.0 / orc.f64("orc_stopping_restricted", x), 1.0, e[i],
                             limit=400, epsrel=1e-12)[0]
        assert R[i] == pytest.approx(ref, rel=1e-9), i
    # grid is uniform in ln E
    assert np.allclose(np.diff(np.log(e)), math.log(300.0) / 1023, rtol=1e-12)


def test_interpolation_is_linear_in_lnE_and_inverse_is_exact(orc):
    t = orc.tables()
    e = np.array(t.e)
    R = np.array(t.R)
    rng = np.random.default_rng(0)
    for _ in range(200):
        i = int(rng.integers(0, 1023))
        f = float(rng.random())
        E = math.exp(math.log(e[i]) + f * (math.log(e[i + 1]) - math.log(e[i])))
        want = R[i] + f * (R[i + 1] - R[i])
        got = orc.f64("orc_range", E)
        assert got == pytest.approx(want, rel=1e-11, abs=1e-14)
        assert orc.f64("orc_range_inverse", got) == pytest.approx(E, rel=1e-11)
    assert orc.f64("orc_range_inverse", 0.0) == 1.0


def test_highland_matches_pdg_formula(orc):
    """theta0 = 13.6 MeV / (beta c p) sqrt(x/X0) [1 + 0.038 ln(x / (X0 beta^2))]."""
    X0 = 36.08
    for E in (70.0, 150.0, 230.0):
        beta2, _ = kin(E)
        pc = math.sqrt(E * E + 2 * E * MP)
        bcp = math.sqrt(beta2) * pc
        for L in (0.5, 1.0, 5.0, 10.0):
            th0 = 13.6 / bcp * math.sqrt(L / X0) * (1 + 0.038 * math.log(L / (X0 * beta2)))
            assert math.sqrt(orc.f64("orc_highland_theta2", E, L)) == pytest.approx(th0, rel=1e-12)
    assert orc.f64("orc_highland_theta2", 150.0, 0.0) == 0.0


def _rocrand_reference(inputs):
    exe = "/tmp/pmc_philox_rocrand"
    if not os.path.exists(exe):
        hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
        subprocess.run([hipcc, "-O1", "-o", exe, os.path.join(HERE, "pins", "philox_rocrand.cpp")],
                       check=True, cwd="/tmp", capture_output=True)
    txt = "\n".join(" ".join(str(int(v)) for v in row) for row in inputs) + "\n"
    out = subprocess.run([exe], input=txt, capture_output=True, text=True, check=True).stdout
    return [list(map(int, l.split())) for l in out.strip().splitlines()]


def test_philox_matches_rocrand(orc):
    """The oracle's Philox4x32-10 against rocRAND's engine (third-party code)."""
    if not (shutil.which("hipcc") or os.path.exists("/opt/rocm/bin/hipcc")):
        pytest.skip("hipcc not available to build the rocRAND reference")
    rng = np.random.default_rng(123)
    rows = [[0, 0, 0, 0, 0, 0], [0xFFFFFFFF] * 6, [1, 2, 3, 0, 7, 0]]
    rows += [list(map(int, rng.integers(0, 2**32, size=6, dtype=np.uint64))) for _ in range(200)]
    ref = _rocrand_reference(rows)
    for row, want in zip(rows, ref):
        got = orc.philox(row[:4], row[4:])
        assert list(map(int, got)) == want, row


def test_delta_sampler_spectrum(orc):
    """KS test of sampled delta energies against the PDG spectrum's CDF, and
    the mean energy per unit path mu_delta <T> = S - L."""
    E = 150.0
    beta2, tmax = kin(E)
    n = 200_000
    T = np.sort(orc.sample_delta(E, n, seed=11))
    assert T.min() >= TCUT and T.max() <= tmax
    norm = integrate.quad(lambda t: spectrum(t, beta2, tmax), TCUT, tmax, epsrel=1e-12)[0]
    grid = np.linspace(TCUT, tmax, 2001)
    cdf = np.array([integrate.quad(lambda t: spectrum(t, beta2, tmax), TCUT, g, epsrel=1e-10)[0]
                    for g in grid]) / norm
    emp = np.searchsorted(T, grid, side="right") / n
    D = np.max(np.abs(emp - cdf))
    assert D < 1.63 / math.sqrt(n) * 1.2, D  # ~1 % level of the KS distribution
    S = orc.f64("orc_stopping_unrestricted", E)
    L = orc.f64("orc_stopping_restricted", E)
    mean_loss = orc.f64("orc_mu_delta", E) * T.mean()
    se = orc.f64("orc_mu_delta", E) * T.std() / math.sqrt(n)
    assert abs(mean_loss - (S - L)) < 4 * se
