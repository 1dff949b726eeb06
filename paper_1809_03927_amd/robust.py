"""Robust-optimisation workload on one GPU.

An optimiser of 4D-robust plans (the future use of Sec. 4.C) needs, for every
breathing phase and every uncertainty scenario, the dose of the whole plan,
and, for the nominal scenario, the dose of every spot separately (the
influence matrix over which it optimises spot weights).  Here: the 4D
thorax phantom, 10 phases x 9 scenarios (nominal, setup shifts of +-3 mm
along x, y and z applied as beam translations, stopping-power ratios scaled
by +-3.5 %) of a 3-field, 8000-spot plan, every calculation with all spots on
one phase; 90 dose calculations sent through the serving loop at once, then
the 1 % influence matrix of the nominal scenario on each phase.

The plain comparison runs the same 90 calculations one after the other with
the plain engine; both must give bit-identical doses.
"""
from __future__ import annotations

import argparse
import json
import sys
import time
from typing import Dict, List

from . import serve as S
from . import workloads as W

RSP_SCALES = (1.0, 1.035, 0.965)


def build(shape_xyz=(256, 256, 160), n_phases=10):
    """Phantoms keyed (calibration index, phase) and plans keyed by shift."""
    base = [W.make_thorax(shape_xyz, p, n_phases) for p in range(n_phases)]
    phantoms = {}
    for ci, scale in enumerate(RSP_SCALES):
        for p, ph in enumerate(base):
            phantoms[(ci, p)] = ph if scale == 1.0 else W.scaled_calibration(ph, scale)
    plans = {}
    for name, shift, _ in W.ROBUST_SCENARIOS:
        plans[name] = W.plan_robust(5, shift_mm=shift)
    return phantoms, plans


def calculations(phantoms, plans, n_phases: int, n_histories: int):
    """(jobs, plan per job): one job per (scenario, phase), all arriving at 0."""
    jobs: List[S.Job] = []
    per_job: Dict[int, W.Plan] = {}
    for si, (name, shift, scale) in enumerate(W.ROBUST_SCENARIOS):
        ci = RSP_SCALES.index(scale)
        for p in range(n_phases):
            i = si * n_phases + p
            key = (ci, p)
            jobs.append(S.Job(i, 0.0, n_histories, key, phantoms[key].nvox))
            per_job[i] = plans[name]
    return jobs, per_job


def influence_nominal(ctx, phantoms, plan: W.Plan, n_phases: int, n_histories: int,
                      rel_threshold=0.01, log=None):
    """Nominal-scenario influence matrix of every phase (each left in the
    context until the next one replaces it); returns per-phase statistics."""
    import torch
    from . import pmc
    stats = []
    slot = 900
    for p in range(n_phases):
        pmc.pmc_load_phase(ctx, slot, phantoms[(0, p)])
        sp = plan.spots.copy()
        sp["phase"] = slot
        pmc.pmc_load_plan(ctx, slot, plan.fields, sp)
        req = pmc.Request(n_histories, [slot], request_id=p, engine=pmc.PMC_ENGINE_PERSISTENT, plan=slot)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nnz, bal, outside = pmc.pmc_influence(ctx, req, None, rel_threshold)
        dt = time.perf_counter() - t0
        if bal["deposited"] + outside + bal["escaped"] + bal["nuclear"] != bal["incident"]:
            raise RuntimeError(f"phase {p}: influence energy balance broken")
        deposited_total = bal["deposited"] + outside
        stats.append({"phase": p, "seconds": dt, "nnz": nnz, "nnz_per_spot": nnz / len(sp),
                      "outside_fraction": outside / max(deposited_total, 1),
                      "histories_per_s": n_histories / dt})
        if log:
            log(f"influence phase {p}: {dt * 1e3:.0f} ms, {nnz} entries "
                f"({nnz / len(sp):.0f} per spot), outside {outside / max(deposited_total, 1):.2e}")
    pmc.pmc_influence_free(ctx)
    pmc.pmc_unload_plan(ctx, slot)
    pmc.pmc_unload_phase(ctx, slot)
    return stats


def run(n_histories=20_000_000, shape_xyz=(256, 256, 160), n_phases=10, depth=1, policy="small-first",
        budget_bytes=0, log=None, plain=True, influence=True, slice_histories=None, n_streams=1,
        launch=None):
    import torch
    from . import pmc
    t0 = time.time()
    phantoms, plans = build(shape_xyz, n_phases)
    if log:
        log(f"built {len(phantoms)} phantoms and {len(plans)} plans in {time.time() - t0:.1f} s")
    free, _ = torch.cuda.mem_get_info()
    budget = int(budget_bytes or 0.9 * free)
    ctx = pmc.pmc_create(0, pmc.PMC_FP32, 5, budget)
    out = {"calculations": len(W.ROBUST_SCENARIOS) * n_phases, "histories_per_calculation": n_histories,
           "spots": int(len(plans["nominal"].spots)), "grid": list(shape_xyz), "budget_bytes": budget}
    try:
        jobs, per_job = calculations(phantoms, plans, n_phases, n_histories)
        engines = [("batched", pmc.PMC_ENGINE_PERSISTENT, policy, depth)]
        if plain:
            engines.append(("plain-serial", pmc.PMC_ENGINE_PLAIN, "fifo", 1))
        digests = {}
        for label, engine, pol, d in engines:
            persistent = engine == pmc.PMC_ENGINE_PERSISTENT
            ex = S.GpuExecutor(ctx, phantoms, per_job, engine, launch if persistent else {},
                               n_streams=n_streams if persistent else 1)
            # every calculation arrives at once and has the same size: no
            # request gains from being cut, so by default each runs whole
            sched = S.Scheduler(ex, S.WallClock(), budget, policy=pol, depth=d, log=log,
                                slice_histories=slice_histories or n_histories)
            done = sched.run([S.Job(j.index, 0.0, j.n_histories, j.phantom_key, j.nvox) for j in jobs])
            ex.close()
            for key in list(ex.slot_of):
                ex.unload_phantom(key)
            s = S.summarize(done, label)
            s.update(slices=sched.slices, peak_bytes=sched.peak_used)
            out[label] = s
            digests[label] = ex.digests
            if log:
                log(f"{label}: {s['makespan_s']:.2f} s for {s['requests']} calculations, "
                    f"{s['throughput_hist_per_s']:.3g} histories/s")
        if plain:
            a, b = digests["batched"], digests["plain-serial"]
            out["identical_doses"] = int(sum(a[k] == b.get(k) for k in a))
        if influence:
            stats = influence_nominal(ctx, phantoms, plans["nominal"], n_phases, n_histories, log=log)
            out["influence"] = {
                "rel_threshold": 0.01, "phases": stats,
                "total_seconds": sum(x["seconds"] for x in stats),
                "total_nnz": sum(x["nnz"] for x in stats),
                "histories_per_s": n_histories * n_phases / sum(x["seconds"] for x in stats)}
        return out
    finally:
        pmc.pmc_destroy(ctx)


def main():
    p = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    p.add_argument("--histories", type=int, default=20_000_000)
    p.add_argument("--phases", type=int, default=10)
    p.add_argument("--grid", type=str, default="256,256,160")
    p.add_argument("--no-plain", action="store_true")
    p.add_argument("--no-influence", action="store_true")
    p.add_argument("--slice-histories", type=int, default=0, help="0 = whole calculations")
    p.add_argument("--streams", type=int, default=1)
    p.add_argument("--tally-mode", choices=["auto", "lane", "core"], default="auto",
                   help="persistent-engine tally mode (auto: the library's choice)")
    a = p.parse_args()
    res = run(a.histories, tuple(int(x) for x in a.grid.split(",")), a.phases, plain=not a.no_plain,
              influence=not a.no_influence, slice_histories=a.slice_histories or None,
              n_streams=a.streams, launch={"tally_mode": ["auto", "lane", "core"].index(a.tally_mode)},
              log=lambda m: print("[robust]", m, file=sys.stderr, flush=True))
    print(json.dumps(res))


if __name__ == "__main__":
    main()
