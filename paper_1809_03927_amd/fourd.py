"""The 4D dose calculation (Sec. 2) on one GPU, trial by trial.

1. Beam-delivery simulation of every trial at once (Sec. 2.B,
   pmc_delivery_simulate): the MU of every spot per breathing phase.
2. Per trial, the sub-plans as one plan (pmc_load_subplans): every (spot,
   phase) that received MU becomes a spot of that phase weighted by that MU
   (Sec. 2.B: the weighting between phases comes from the delivery, Eq. (2)
   adds no other).
3. The Monte Carlo dose of all phases in one batched persistent launch
   (Sec. 2.C, pmc_dose_device): histories split over the sub-plan spots in
   proportion to MU.
4. Deformable accumulation onto the reference phase (Sec. 2.D.2,
   pmc_accumulate_device / pmc_accumulate_dim_device).

The trials are the delivery-uncertainty study of Sec. 2.B (start phase,
breathing period, synchrotron parameters drawn per trial).  PyTorch owns the
device buffers and the stream; every step runs in libpmc.  Trials are
pipelined: the host loads trial i+1's sub-plans and prepares its work items
while the device still runs trial i (everything is enqueued on one stream,
so trial i's accumulation has read the tallies before trial i+1 clears
them); the host waits only at the end.
"""
from __future__ import annotations

import time
from typing import Optional, Sequence

import numpy as np

from . import pmc


class FourD:
    """A 4D dose calculation on a context whose phases (and DVFs) are loaded.

    phase_ids[p]: the loaded phase of breathing phase p; ref: index of the
    reference (accumulation) phase in phase_ids; dvf_ids[p]: the loaded DVF
    of phase p (source -> reference for EMTM, reference -> source for DIM;
    ignored for the reference); nvox: voxels per phase (one grid for all)."""

    def __init__(self, ctx, fields: np.ndarray, spots: np.ndarray, phase_ids: Sequence[int], ref: int,
                 dvf_ids: Sequence[Optional[int]], nvox: int, n_sub: int = 5, method: str = "emtm",
                 plan_id: int = 900, tally_mode: int = pmc.PMC_TALLY_AUTO):
        import torch
        if method not in ("emtm", "dim"):
            raise ValueError("method must be 'emtm' or 'dim'")
        self.ctx, self.fields, self.spots = ctx, fields, spots
        self.phase_ids = [int(p) for p in phase_ids]
        self.ref, self.n_sub, self.method, self.plan_id = ref, n_sub, method, plan_id
        self.src = [p for p in range(len(self.phase_ids)) if p != ref]
        self.dvf_ids = [int(dvf_ids[p]) for p in self.src]
        self.nvox = nvox
        self.tally_mode = tally_mode
        self.torch = torch
        self.stream = torch.cuda.Stream()
        dev = torch.device("cuda")
        self.tallies = [torch.zeros(nvox, dtype=torch.int64, device=dev) for _ in self.phase_ids]
        self.counters = torch.zeros(pmc.PMC_COUNTERS, dtype=torch.int64, device=dev)
        self.dose = torch.zeros(nvox, dtype=torch.float64, device=dev)
        self.mask = torch.zeros(nvox, dtype=torch.uint8, device=dev)

    def run(self, delivery, n_histories: int, request_id: int = 0, keep: bool = True) -> dict:
        """All trials of `delivery`; returns the accumulated doses (host, Gy
        per history of each trial's run) if keep, the report mask, the
        delivery result, the wall time of the delivery call and of the whole
        loop, and per trial the host time to load and enqueue it and the
        device times of its Monte Carlo and accumulation (events)."""
        torch = self.torch
        st = self.stream
        t0 = time.perf_counter()
        dl = pmc.pmc_delivery_simulate(self.ctx, delivery, self.spots, len(self.fields))
        t_delivery = time.perf_counter() - t0
        kept, t_host, events = [], [], []
        tptr = [t.data_ptr() for t in self.tallies]
        acc = pmc.pmc_accumulate_device if self.method == "emtm" else pmc.pmc_accumulate_dim_device
        t_loop = time.perf_counter()
        for trial in range(delivery.n_trials):
            t1 = time.perf_counter()
            pmc.pmc_load_subplans(self.ctx, self.plan_id, self.fields, self.spots, dl["mu"][trial],
                                  self.phase_ids)
            req = pmc.Request(n_histories, self.phase_ids, request_id=request_id + trial,
                              engine=pmc.PMC_ENGINE_PERSISTENT, plan=self.plan_id, tally_mode=self.tally_mode)
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            with torch.cuda.stream(st):
                for t in self.tallies:
                    t.zero_()
                self.counters.zero_()
                ev[0].record(st)
            pmc.pmc_dose_device(self.ctx, req, st.cuda_stream, tptr, self.counters.data_ptr())
            ev[1].record(st)
            acc(self.ctx, self.phase_ids[self.ref], tptr[self.ref], [self.phase_ids[p] for p in self.src],
                self.dvf_ids, [tptr[p] for p in self.src], self.n_sub, n_histories, st.cuda_stream,
                self.dose.data_ptr(), self.mask.data_ptr())
            ev[2].record(st)
            if keep:
                with torch.cuda.stream(st):
                    host = torch.empty(self.nvox, dtype=torch.float64, pin_memory=True)
                    host.copy_(self.dose, non_blocking=True)
                kept.append(host)
            events.append(ev)
            t_host.append(time.perf_counter() - t1)
        st.synchronize()
        total = time.perf_counter() - t_loop
        return {"doses": [h.numpy() for h in kept], "mask": self.mask.cpu().numpy().astype(bool), "delivery": dl,
                "time_delivery_s": t_delivery, "time_loop_s": total, "time_host_s": t_host,
                "time_mc_s": [e[0].elapsed_time(e[1]) * 1e-3 for e in events],
                "time_accumulation_s": [e[1].elapsed_time(e[2]) * 1e-3 for e in events]}

    def close(self):
        try:
            pmc.pmc_unload_plan(self.ctx, self.plan_id)
        except pmc.PmcError:
            pass


def dvh(dose: np.ndarray, roi: np.ndarray, bins: np.ndarray) -> np.ndarray:
    """Cumulative dose-volume histogram: fraction of the ROI's voxels
    receiving at least each bin dose."""
    d = np.asarray(dose)[np.asarray(roi, dtype=bool).ravel()]
    if d.size == 0:
        return np.zeros(len(bins))
    return np.array([(d >= b).mean() for b in bins])
