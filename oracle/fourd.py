"""The 4D dose calculation composed from the oracle's parts, FP64.

TEST INFRASTRUCTURE ONLY (like the rest of `oracle/`): imported by tests,
never by the product package.

Sec. 2 of the paper chains three steps: the beam-delivery simulation
(Sec. 2.B, `oracle.delivery`) gives the MU of every spot per breathing
phase; each phase's sub-plan is the spots delivered in it with that MU as
weight (the reading used with the library: spot order, then phase;
histories split over the sub-plan spots in proportion to MU); the Monte
Carlo (Sec. 2.C, `oracle.dose`) gives the tally of every phase; the
energy/mass-transfer accumulation (Sec. 2.D.2, Eqs. (2), (4)-(6),
`oracle.emtm`) puts them on the reference phase.  One accumulated dose per
delivery trial, in Gy per history of that trial's run.
"""
from __future__ import annotations

import numpy as np

import oracle
from oracle import delivery as DL
from oracle import emtm as EM
from paper_1809_03927_amd.workloads import Plan


def sub_plan(spots: np.ndarray, mu: np.ndarray) -> np.ndarray:
    """Plan spots of one delivery: for each spot s in order and each phase p
    in order, spot s on phase p weighted by its MU there, if any."""
    rows = []
    for s in range(len(spots)):
        for p in range(mu.shape[1]):
            if mu[s, p] > 0.0:
                r = spots[s].copy()
                r["phase"] = p
                r["weight"] = mu[s, p]
                rows.append(r)
    return np.array(rows, dtype=spots.dtype)


def densities(phases):
    return [oracle.convert(ph, np.zeros(ph.hu.size, dtype=np.int64), 1)[1] for ph in phases]


def fourd(phases, fields, spots, delivery, ref: int, dvfs, n_sub: int, n_hist: int, seed: int,
          request_id: int = 0, n_batches: int = 0, n_threads=None):
    """Every trial of `delivery` on `phases` (breathing phase p = phases[p]);
    dvfs[p] maps phase p to the reference (None for the reference).  Returns
    the delivery result and per trial the accumulated dose (request id
    request_id + trial), and with n_batches > 0 also the accumulated dose of
    each history batch (history index mod n_batches) -- Eq. (5) is linear in
    the energies for fixed masses, so the batches sum to the whole."""
    dl = DL.simulate(spots, len(fields), delivery)
    rho = densities(phases)
    out, batches = [], []
    for trial in range(delivery.n_trials):
        plan = Plan(fields, sub_plan(spots, dl["mu"][trial]))
        rid = request_id + trial
        tallies, _, _ = oracle.dose(phases, plan, n_hist, seed, rid, with_dose=False, n_threads=n_threads)
        out.append(EM.emtm(phases, tallies, rho, ref, dvfs, n_sub, n_hist)["dose"])
        if n_batches:
            bt = []
            for b in range(n_batches):
                t, _ = oracle.dose_subset(phases, plan, n_hist, seed, 0, 2**32 - 1, rid, n_threads=n_threads,
                                          h_mod=n_batches, h_rem=b)
                bt.append(EM.emtm(phases, t, rho, ref, dvfs, n_sub, n_hist)["dose"])
            batches.append(bt)
    return dl, out, batches
