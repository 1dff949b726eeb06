"""Beam-delivery simulation (Sec. 2.B, App. A): the oracle
(`oracle.delivery`) against hand-computed timelines (fixed parameters),
closed forms for synchrotron refills, gating and repainting, and invariants
(MU conservation, no beam outside the gate window, the draws' moments and
ranges)."""
import numpy as np
import pytest

from paper_1809_03927_amd import workloads as W

DL = pytest.importorskip("oracle.delivery")


def spots(rows):
    """rows: (energy, x, y, MU, field)."""
    out = np.zeros(len(rows), dtype=W.SPOT_DTYPE)
    for i, (e, x, y, mu, f) in enumerate(rows):
        out[i]["energy_MeV"] = e
        out[i]["x_mm"] = x
        out[i]["y_mm"] = y
        out[i]["sigma_mm"] = 5.0
        out[i]["weight"] = mu
        out[i]["field"] = f
    return out


def fixed(switch=2.0, discard=0.07, rate=10.0, spot_switch=0.01, per_mm=0.0, capacity=100.0, tmax=8.0):
    return {"layer_switch_s": (switch, 0.0), "layer_switch_per_mev": (0.0, 0.0), "discard_s": (discard, 0.0),
            "spill_rate_mu_s": (rate, 0.0), "spill_rate_per_mev": (0.0, 0.0),
            "spot_switch_s": (spot_switch, 0.0), "spot_switch_per_mm": (per_mm, 0.0),
            "capacity_mu": (capacity, 0.0), "extraction_max_s": (tmax, 0.0)}


def phases_of(mu):
    return [int(np.flatnonzero(row)[0]) for row in mu]


def test_hand_computed_timeline():
    """N = 10 phases of 0.4 s from phase 0.  Layer 1 (70 MeV, MU 1, 2, 3):
    switch 2 s + discard 0.07 -> spots start at 2.07, 2.18, 2.39 (phase 5),
    ending 2.69; layer 2 (100 MeV, MU 1, 1): 4.69 + 0.07 -> starts at 4.76
    (phase 11 -> 1) and 4.87 (phase 12 -> 2), ending at 4.97."""
    sp = spots([(70.0, 0, 0, 1.0, 0), (70.0, 5, 0, 2.0, 0), (70.0, 10, 0, 3.0, 0),
                (100.0, 0, 0, 1.0, 0), (100.0, 5, 0, 1.0, 0)])
    d = W.Delivery(n_phases=10, start_phase=0, period_s=4.0, sync=fixed())
    out = DL.simulate(sp, 1, d)
    assert phases_of(out["mu"][0]) == [5, 5, 5, 1, 2]
    assert np.allclose(out["mu"][0].sum(axis=1), [1, 2, 3, 1, 1], rtol=0, atol=0)
    assert out["time"][0, 0] == pytest.approx(4.97, abs=1e-12)
    assert out["fills"][0, 0] == 2


def test_capacity_refills():
    """10 spots of 1 MU, 3 MU per fill: fills of 3, 3, 3, 1 spots; every
    spot switch counts, and each new fill costs a layer switch and a discard:
    T = 4 S + 4 D + 10 x 0.1 + 9 w."""
    sp = spots([(120.0, 2.0 * i, 0, 1.0, 0) for i in range(10)])
    S, Dd, w = 1.5, 0.07, 0.004
    d = W.Delivery(n_phases=10, start_phase=0, period_s=4.0,
                   sync=fixed(switch=S, discard=Dd, rate=10.0, spot_switch=w, capacity=3.0))
    out = DL.simulate(sp, 1, d)
    assert out["fills"][0, 0] == 4
    assert out["time"][0, 0] == pytest.approx(4 * S + 4 * Dd + 1.0 + 9 * w, abs=1e-12)


def test_extraction_time_limit():
    """Spills of 1 s each (10 MU at 10 MU/s) and a 2.5 s extraction limit:
    two spots per fill (the third would end at 2 + w + 1 > 2.5 s)."""
    sp = spots([(150.0, 0, 0, 10.0, 0) for _ in range(5)])
    S, Dd, w = 1.0, 0.07, 0.01
    d = W.Delivery(n_phases=10, start_phase=0, period_s=4.0,
                   sync=fixed(switch=S, discard=Dd, rate=10.0, spot_switch=w, tmax=2.5))
    out = DL.simulate(sp, 1, d)
    assert out["fills"][0, 0] == 3
    assert out["time"][0, 0] == pytest.approx(3 * S + 3 * Dd + 5.0 + 4 * w, abs=1e-12)


def test_gate_waits_for_the_window():
    """Gate on phases 3-5 (0.4 s each from phase 0): the first fill waits
    from 0.5 s until phase 3 starts at 1.2 s; spots of 0.5 s run 1.27-1.77,
    1.78-2.28, then the third starts at 2.29 (phase 5), the fourth would
    start at 2.80 (phase 7): it waits for the next phase 3 at 5.2 s and
    discards beam again (5.27)."""
    sp = spots([(100.0, 0, 0, 5.0, 0) for _ in range(4)])
    d = W.Delivery(n_phases=10, start_phase=0, period_s=4.0, gate_lo=3, gate_hi=5,
                   sync=fixed(switch=0.5, discard=0.07, rate=10.0, spot_switch=0.01))
    out = DL.simulate(sp, 1, d)
    assert phases_of(out["mu"][0]) == [3, 4, 5, 3]
    assert out["time"][0, 0] == pytest.approx(5.27 + 0.5, abs=1e-12)


def test_isolayered_repainting_pieces():
    """max 0.4 MU per delivery: MU 1.0 -> 0.4, 0.4, 0.2; 0.3 -> 0.3;
    0.8 -> 0.4, 0.4: six deliveries in one fill."""
    sp = spots([(90.0, 0, 0, 1.0, 0), (90.0, 4, 0, 0.3, 0), (90.0, 8, 0, 0.8, 0)])
    S, Dd, w = 2.0, 0.07, 0.002
    d = W.Delivery(n_phases=1, start_phase=0, period_s=4.0, max_mu=0.4,
                   sync=fixed(switch=S, discard=Dd, rate=10.0, spot_switch=w))
    out = DL.simulate(sp, 1, d)
    assert np.allclose(out["mu"][0][:, 0], [1.0, 0.3, 0.8], rtol=1e-15)
    assert out["time"][0, 0] == pytest.approx(S + Dd + 2.1 / 10.0 + 5 * w, abs=1e-12)


def test_random_trials_conserve_mu_and_respect_the_gate():
    plan = W.plan_thorax(3, n_phases=10)
    sp = plan.spots.copy()
    sp["weight"] = sp["weight"] / sp["weight"].sum() * 200.0
    sp = sp[:600]
    d = W.Delivery(n_trials=4, period_sd_s=0.5, period_min_s=3, period_max_s=7, gate_lo=3, gate_hi=7,
                   max_mu=0.05, seed=9)
    out = DL.simulate(sp, 1, d)
    assert np.allclose(out["mu"].sum(axis=2), np.broadcast_to(sp["weight"], (4, len(sp))), rtol=1e-12)
    assert not out["mu"][:, :, [0, 1, 2, 8, 9]].any()
    assert out["mu"][:, :, 3:8].sum() > 0
    # the trials differ (start phase, period, synchrotron draws)
    assert len({float(t) for t in out["time"][:, 0]}) == 4


def test_draws():
    """The delivery Gaussians are N(0, 1) (Sec. 2.B, App. A: N(mu, sigma)):
    Kolmogorov-Smirnov against scipy's normal CDF, the fourth moment (3 for a
    normal; the 12-uniform sum this replaced has 2.9, six standard errors
    away at this sample size) and the tail beyond 3 sigma; |z| <= 6.77 (the
    smallest uniform is 2^-33).  Start phases and periods cover their ranges."""
    from scipy import stats
    key = [5, 2]
    z = np.array([DL.gauss(key, f, 2, k) for f in range(4) for k in range(25000)])
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(z.mean()) < 0.02 and abs(z.var() - 1.0) < 0.02
    kurt = np.mean(z ** 4) / np.mean(z ** 2) ** 2
    assert abs(kurt - 3.0) < 0.06, kurt
    tail = np.mean(np.abs(z) > 3.0)
    assert abs(tail - 2 * stats.norm.sf(3.0)) < 4 * np.sqrt(2.7e-3 / len(z)), tail
    assert np.abs(z).max() <= np.sqrt(66 * np.log(2.0))
    starts = {DL.draw_int([s, 0], 0, DL.P_START, 10) for s in range(200)}
    assert starts == set(range(10))
    periods = {3 + DL.draw_int([s, 0], 0, DL.P_PERIOD, 5) for s in range(200)}
    assert periods == {3, 4, 5, 6, 7}


def test_margin_logs_near_ties():
    """The oracle's margin is the smallest relative gap of a decision a
    last-bit difference could flip.  Hand timeline with a 2.05 s layer
    switch (phases of 0.4 s from phase 0): the first fill's gate check at
    2.05, starts 2.12, 2.23, 2.44 (phase 6), end 2.74; the second layer's
    check at 4.79, 0.01 s before the boundary at 4.8 -- the smallest gap,
    0.01 / 4.8 -- then starts 4.86 and 4.97.  A switch that ends exactly on
    a boundary logs 0, one that ends 1e-13 s before it logs below 1e-12."""
    sp = spots([(70.0, 0, 0, 1.0, 0), (70.0, 5, 0, 2.0, 0), (70.0, 10, 0, 3.0, 0),
                (100.0, 0, 0, 1.0, 0), (100.0, 5, 0, 1.0, 0)])
    d = W.Delivery(n_phases=10, start_phase=0, period_s=4.0, sync=fixed(switch=2.05))
    out = DL.simulate(sp, 1, d)
    assert phases_of(out["mu"][0]) == [5, 5, 6, 2, 2]
    assert out["time"][0, 0] == pytest.approx(5.07, abs=1e-12)
    assert out["margin"][0, 0] == pytest.approx(0.01 / 4.8, rel=1e-9)
    on = DL.simulate(sp[:1], 1, W.Delivery(n_phases=10, start_phase=0, period_s=4.0, sync=fixed(switch=2.0)))
    assert on["margin"][0, 0] < 1e-15
    near = DL.simulate(sp[:1], 1, W.Delivery(n_phases=10, start_phase=0, period_s=4.0,
                                             sync=fixed(switch=2.0 - 1e-13)))
    assert 0 < near["margin"][0, 0] < 1e-12
