"""Beam-delivery simulation on the GPU (pmc_delivery_simulate, through the C
ABI) against the oracle (`oracle.delivery`): the same Philox draws and the
same FP64 operations in the same order; the Box-Muller logarithm and cosine
are the device's and the host's, so MU per phase and fill counts are
identical and end times agree to 1e-12 except in a timeline with a decision
at a near tie (logged by the oracle; see `delivery_check`)."""
import sys

import numpy as np
import pytest

from delivery_check import compare, same
from paper_1809_03927_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def P():
    from paper_1809_03927_amd import pmc
    return pmc


@pytest.fixture(scope="module")
def DL():
    import oracle.delivery as dl
    return dl


def run(P, d, sp, n_fields):
    ctx = P.pmc_create(0, P.PMC_FP32, 1, 0)
    try:
        return P.pmc_delivery_simulate(ctx, d, sp, n_fields)
    finally:
        P.pmc_destroy(ctx)


def test_hand_computed_timeline(P, DL):
    sp = np.zeros(5, dtype=W.SPOT_DTYPE)
    sp["energy_MeV"] = [70.0, 70.0, 70.0, 100.0, 100.0]
    sp["x_mm"] = [0, 5, 10, 0, 5]
    sp["weight"] = [1.0, 2.0, 3.0, 1.0, 1.0]
    sync = {k: (v, 0.0) for k, v in dict(layer_switch_s=2.0, layer_switch_per_mev=0.0, discard_s=0.07,
                                         spill_rate_mu_s=10.0, spill_rate_per_mev=0.0, spot_switch_s=0.01,
                                         spot_switch_per_mm=0.0, capacity_mu=100.0,
                                         extraction_max_s=8.0).items()}
    d = W.Delivery(n_phases=10, start_phase=0, period_s=4.0, sync=sync)
    say("delivery hand timeline")
    got = run(P, d, sp, 1)
    assert got["time"][0, 0] == pytest.approx(4.97, abs=1e-12)
    assert [int(np.flatnonzero(r)[0]) for r in got["mu"][0]] == [5, 5, 5, 1, 2]
    # every standard deviation is 0: no draw reaches the timeline
    same(got, {k: v for k, v in DL.simulate(sp, 1, d).items() if k != "margin"})


@pytest.mark.parametrize("mode", ["free", "gated", "repainted"])
def test_random_trials_match_oracle(P, DL, mode):
    """The thorax plan (3000 spots, 20 layers, one field), 6 trials with random
    start phase, period U{3..7} s, sigma 0.4 s and synchrotron uncertainty;
    free breathing, gated on phases 3-7, or repainted at 0.005 MU (the
    paper's three delivery scenarios)."""
    plan = W.plan_thorax(3, n_phases=10)
    sp = plan.spots.copy()
    sp["weight"] = sp["weight"] / sp["weight"].sum() * 250.0
    kw = dict(n_trials=6, period_sd_s=0.4, period_min_s=3, period_max_s=7, seed=21)
    if mode == "gated":
        kw.update(gate_lo=3, gate_hi=7)
    if mode == "repainted":
        kw.update(max_mu=0.005)
    d = W.Delivery(**kw)
    say("delivery random trials", mode)
    got = run(P, d, sp, len(plan.fields))
    want = DL.simulate(sp, len(plan.fields), d)
    compare(got, want, sp, len(plan.fields), max_flips=1)
    assert np.allclose(got["mu"].sum(axis=2), np.broadcast_to(sp["weight"], (6, len(sp))), rtol=1e-12)


def test_three_fields(P, DL):
    """The robust plan's three fields (8000 spots) in 4 trials: one thread per
    (trial, field), fields interleaved in the spot array are kept apart."""
    plan = W.plan_robust()
    sp = plan.spots.copy()
    sp["weight"] = sp["weight"] / sp["weight"].sum() * 600.0
    # interleave the fields in the array (each field keeps its own order)
    per = [np.flatnonzero(sp["field"] == f) for f in range(len(plan.fields))]
    order = [i for k in range(max(len(x) for x in per)) for x in per if k < len(x) for i in [x[k]]]
    sp = sp[np.array(order)]
    assert sp["field"][0] != sp["field"][1]
    d = W.Delivery(n_trials=4, period_sd_s=0.3, gate_lo=2, gate_hi=6, max_mu=0.02, seed=5)
    say("delivery three fields")
    got = run(P, d, sp, len(plan.fields))
    compare(got, DL.simulate(sp, len(plan.fields), d), sp, len(plan.fields), max_flips=1)


def test_degenerate_deliveries(P, DL):
    """A field without spots, a single breathing phase, a gate open on every
    phase (the same as free breathing), max_MU above every spot's MU (the
    same as no repainting), and an empty plan."""
    plan = W.plan_thorax(3, n_phases=10)
    sp = plan.spots.copy()[:400]
    sp["weight"] = sp["weight"] / sp["weight"].sum() * 40.0
    base = dict(n_trials=3, period_sd_s=0.3, seed=4)
    say("delivery: empty second field")
    got = run(P, W.Delivery(**base), sp, 2)
    want = DL.simulate(sp, 2, W.Delivery(**base))
    compare(got, want, sp, 2, max_flips=1)
    assert not got["time"][:, 1].any() and not got["fills"][:, 1].any()
    say("delivery: one phase")
    one = run(P, W.Delivery(n_phases=1, **base), sp, 1)
    assert np.array_equal(one["mu"][:, :, 0], np.broadcast_to(sp["weight"], (3, len(sp))))
    say("delivery: gate on every phase, max MU above every spot")
    free = run(P, W.Delivery(**base), sp, 1)
    gated_all = run(P, W.Delivery(gate_lo=0, gate_hi=9, **base), sp, 1)
    big = run(P, W.Delivery(max_mu=float(sp["weight"].max()) * 2, **base), sp, 1)
    same(gated_all, free)
    same(big, free)
    say("delivery: empty plan")
    empty = run(P, W.Delivery(**base), sp[:0], 1)
    assert empty["mu"].shape == (3, 0, 10) and not empty["time"].any()
