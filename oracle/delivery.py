"""Beam-delivery simulation, plain Python in FP64.

TEST INFRASTRUCTURE ONLY (like the rest of `oracle/`): imported by tests and
by the benchmark's CPU-baseline leg, never by the product package.

Follows Sec. 2.B and App. A of the paper; the readings where it is silent are
those of the library's documentation of pmc_delivery_simulate:

* every (trial, field) is an independent timeline starting at t = 0 at the
  start of breathing phase phi0 (given, or U{0..N-1} per trial and field);
* breathing: the k-th phase occurrence lasts P_k / N with P_k = mu + sigma z_k
  (at least mu / 20); phase occurrence k is phase (phi0 + k) mod N; mu is
  given or U{min..max} seconds per trial and field;
* synchrotron parameters are drawn once per trial and field as
  central + sd z, clipped at 0;
* z ~ N(0, 1) (the paper's N(mu, sigma) draws, Sec. 2.B and App. A) by the
  Box-Muller transform in FP64, z = sqrt(-2 ln u_a) cos(2 pi u_b), from the
  first two words of one Philox block, key (seed mod 2^32, trial), counter
  (field, purpose, index, 0), each word x as u = (x + 1/2) 2^-32;
* a layer is the run of consecutive spots of one field with one energy; each
  layer costs a layer switch a + b (E - 70 MeV); every fill of the synchrotron
  starts by waiting for the gate (gated delivery) and discarding beam;
* deliveries of a layer: painting r gives each spot min(MU - r max_MU,
  max_MU) while positive (no repainting: the whole MU once); between two
  deliveries of a fill the beam is off for e + f max(|dx|, |dy|); a delivery
  that would exceed the fill's charge or extraction time (and is not the
  fill's first) starts a new fill at the same energy (layer switch, gate,
  discard); a delivery that finds the gate closed waits for it and discards
  beam again; the delivery belongs wholly to the breathing phase at its start
  and lasts MU / (c + d (E - 70 MeV)).

The logarithm and cosine are the host's libm, so another implementation of
the same definition (the device's) may differ in the last bit of z.  Every
decision that such a difference could flip is a comparison of two FP64
values; `simulate` records, per (trial, field), the smallest relative gap
|a - b| / max(|a|, |b|) among them (phase boundaries against delivery
times, the fill's charge against the next delivery's MU, the extraction
time against its limit), so that a comparison can tell a last-bit flip at a
near tie from a real difference.
"""
from __future__ import annotations

import math
from typing import Dict

import numpy as np

import oracle
from paper_1809_03927_amd.workloads import SYNC_PARAMS

TWO_M32 = 2.0 ** -32
TWO_PI = 2.0 * math.pi
P_START, P_SYNC, P_BREATH, P_PERIOD = 0, 1, 2, 3


def words(key, field, purpose, index, block):
    return [int(x) for x in oracle.philox([field, purpose, index, block], key)]


def gauss(key, field, purpose, index) -> float:
    """A standard normal deviate by Box-Muller: u = (x + 1/2) 2^-32 of the
    first two words of block 0, z = sqrt(-2 ln u_a) cos(2 pi u_b)."""
    w = words(key, field, purpose, index, 0)
    ua = (w[0] + 0.5) * TWO_M32
    ub = (w[1] + 0.5) * TWO_M32
    return math.sqrt(-2.0 * math.log(ua)) * math.cos(TWO_PI * ub)


def gap(a, b) -> float:
    """Relative gap of a comparison of a with b."""
    m = max(abs(a), abs(b))
    return abs(a - b) / m if m > 0.0 else 0.0


def draw_int(key, field, purpose, n) -> int:
    """U{0..n-1} from the first word of block 0: floor(x n / 2^32)."""
    return (words(key, field, purpose, 0, 0)[0] * n) >> 32


class Breathing:
    """The breathing timeline of one (trial, field)."""

    def __init__(self, key, field, d, phi0, mu):
        self.key, self.field, self.d, self.phi0, self.mu = key, field, d, phi0, mu
        self.k = 0
        self.t0 = 0.0
        self.t1 = self.length(0)
        self.margin = math.inf

    def length(self, k):
        p = self.mu + self.d.period_sd_s * gauss(self.key, self.field, P_BREATH, k)
        if p < self.mu / 20.0:
            p = self.mu / 20.0
        return p / self.d.n_phases

    def phase(self, t, log=True):
        """Phase at time t (t never decreases).  With log, the gaps of the
        comparisons with the boundaries go into the margin; without, t is a
        boundary itself (the gate's opening), an exact comparison."""
        moved = False
        while t >= self.t1:
            if log:
                self.margin = min(self.margin, gap(t, self.t1))
            self.k += 1
            self.t0 = self.t1
            self.t1 = self.t0 + self.length(self.k)
            moved = True
        if log or moved:
            self.margin = min(self.margin, gap(t, self.t1))
        return (self.phi0 + self.k) % self.d.n_phases

    def gated_open(self, ph):
        return self.d.gate_lo < 0 or (self.d.gate_lo <= ph <= self.d.gate_hi)

    def wait_gate(self, t):
        """The first time >= t at which the gate is open."""
        ph = self.phase(t)
        while not self.gated_open(ph):
            t = self.t1
            ph = self.phase(t, log=False)
        return t


def simulate(spots: np.ndarray, n_fields: int, d) -> Dict[str, np.ndarray]:
    """spots: structured array (energy_MeV, x_mm, y_mm, weight = MU, field) in
    delivery order within each field.  Returns mu (n_trials, n_spots, N), the
    end time (n_trials, n_fields) in s, the number of synchrotron fills and
    the smallest relative gap of a decision per (trial, field) ("margin")."""
    n = len(spots)
    N = d.n_phases
    mu_out = np.zeros((d.n_trials, n, N))
    t_out = np.zeros((d.n_trials, n_fields))
    fills_out = np.zeros((d.n_trials, n_fields), dtype=np.int64)
    margin_out = np.full((d.n_trials, n_fields), np.inf)
    gated = d.gate_lo >= 0
    for trial in range(d.n_trials):
        key = [d.seed & 0xFFFFFFFF, trial]
        for field in range(n_fields):
            idx = [i for i in range(n) if int(spots["field"][i]) == field]
            if not idx:
                continue
            par = {}
            for i, name in enumerate(SYNC_PARAMS):
                c, sd = d.sync[name]
                v = c + sd * gauss(key, field, P_SYNC, i)
                par[name] = v if v > 0.0 else 0.0
            phi0 = d.start_phase if d.start_phase >= 0 else draw_int(key, field, P_START, N)
            if 0 < d.period_min_s <= d.period_max_s:
                mean = float(d.period_min_s + draw_int(key, field, P_PERIOD, d.period_max_s - d.period_min_s + 1))
            else:
                mean = d.period_s
            br = Breathing(key, field, d, phi0, mean)
            t = 0.0
            fills = 0
            layers = []
            for i in idx:
                if layers and spots["energy_MeV"][layers[-1][0]] == spots["energy_MeV"][i]:
                    layers[-1].append(i)
                else:
                    layers.append([i])
            for layer in layers:
                e = float(spots["energy_MeV"][layer[0]])
                switch = par["layer_switch_s"] + par["layer_switch_per_mev"] * (e - 70.0)
                rate = par["spill_rate_mu_s"] + par["spill_rate_per_mev"] * (e - 70.0)
                # the synchrotron reaches the layer's energy, then a fill starts
                t = t + switch
                t = br.wait_gate(t) + par["discard_s"]
                t_ext = t
                q = par["capacity_mu"]
                fills += 1
                fresh = True
                prev = None
                r = 0
                while True:
                    any_left = False
                    for i in layer:
                        total = float(spots["weight"][i])
                        if d.max_mu > 0.0:
                            m = total - r * d.max_mu
                            if m > d.max_mu:
                                m = d.max_mu
                        else:
                            m = total if r == 0 else 0.0
                        if m <= 0.0:
                            continue
                        any_left = True
                        x, y = float(spots["x_mm"][i]), float(spots["y_mm"][i])
                        if prev is not None:
                            dx, dy = abs(x - prev[0]), abs(y - prev[1])
                            t = t + (par["spot_switch_s"] + par["spot_switch_per_mm"] * (dx if dx > dy else dy))
                        spill = m / rate
                        if not fresh:
                            br.margin = min(br.margin, gap(m, q),
                                            gap((t - t_ext) + spill, par["extraction_max_s"]))
                        if not fresh and (m > q or (t - t_ext) + spill > par["extraction_max_s"]):
                            t = t + switch
                            t = br.wait_gate(t) + par["discard_s"]
                            t_ext = t
                            q = par["capacity_mu"]
                            fills += 1
                        if gated and not br.gated_open(br.phase(t)):
                            t = br.wait_gate(t) + par["discard_s"]
                        ph = br.phase(t)
                        mu_out[trial, i, ph] = mu_out[trial, i, ph] + m
                        t = t + spill
                        q = q - m
                        fresh = False
                        prev = (x, y)
                    if not any_left:
                        break
                    r += 1
            t_out[trial, field] = t
            fills_out[trial, field] = fills
            margin_out[trial, field] = br.margin
    return {"mu": mu_out, "time": t_out, "fills": fills_out, "margin": margin_out}
