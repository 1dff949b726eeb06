"""Benchmark of the proton dose engine on one MI355X.

One step = one full 4D dose calculation of the thorax workload (10 breathing
phases of 256x256x160 voxels, 3000 spots assigned to phases by the delivery
clock, 5e7 histories): zero the int64 tallies, run the transport of all
phases (one persistent launch: work queue + lane refill; or, for the plain
engine, one launch per phase), and convert every phase's tally to dose.
Inputs (phantoms, tables, plan) are resident on the device before timing.

Prints one JSON line.  `value` is histories/s of the batched (persistent)
engine; the plain engine's rate on the same workload is reported beside it.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X: 256 CUs, 4 SIMD16 units each, 2.4 GHz peak engine clock.  A wave64
# VALU instruction occupies a SIMD for 4 cycles, so the chip issues at most
# 256 * 4 * 16 * 2.4e9 = 3.93e13 full-rate lane operations per second.
PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
HBM_PEAK_GBS = 8000.0

# VALU instructions one lane executes per transport step, measured with the
# SQ_INSTS_VALU counter on single-history launches of the FP32 kernel (see
# profiles/transport_valu_per_step.md).
VALU_PER_STEP = float(os.environ.get("PMC_VALU_PER_STEP", "0") or 0) or None


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--plain-steps", type=int, default=2)
    p.add_argument("--histories", type=int, default=50_000_000)
    p.add_argument("--grid", type=str, default="256,256,160")
    p.add_argument("--chunk", type=int, default=0)
    p.add_argument("--block", type=int, default=0)
    p.add_argument("--refill", type=int, default=0)
    p.add_argument("--no-plain", action="store_true")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--mode", choices=["bench", "single-history"], default="bench")
    return p.parse_args()


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this engine runs on one GPU; multi-GPU sharding is a design "
                                   "note only (see DESIGN.md)", "n_gpus": a.gpus}))
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1809_03927_amd import pmc
    from paper_1809_03927_amd import workloads as W

    grid = tuple(int(x) for x in a.grid.split(","))
    t0 = time.time()
    wl = W.workload_thorax4d(a.histories, shape_xyz=grid)
    log(f"workload {wl.name}: {len(wl.phases)} phases {grid}, {len(wl.plan.spots)} spots, "
        f"spots/phase {np.bincount(wl.plan.spots['phase'], minlength=10).tolist()} "
        f"({time.time() - t0:.1f} s to generate)")
    dev = torch.device("cuda:0")
    eng = pmc.Engine(device=0, precision=pmc.PMC_FP32, seed=wl.seed)
    eng.load_workload(wl)
    phases = list(range(len(wl.phases)))
    nvox = wl.phases[0].nvox
    tallies = [torch.zeros(nvox, dtype=torch.int64, device=dev) for _ in phases]
    doses = [torch.zeros(nvox, dtype=torch.float64, device=dev) for _ in phases]
    counters = torch.zeros(pmc.PMC_COUNTERS, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()

    if a.mode == "single-history":
        # one history per launch: VALU instructions per step of one lane
        req = pmc.Request(1, [0], engine=pmc.PMC_ENGINE_PLAIN, block_size=64)
        one = W.workload_thorax4d(1, shape_xyz=grid)
        one.plan.spots = one.plan.spots[:1].copy()
        one.plan.spots["phase"] = 0
        eng.load_plan(one.plan)
        for _ in range(20):
            counters.zero_()
            pmc.pmc_dose_device(eng.ctx, req, stream.cuda_stream, [tallies[0].data_ptr()],
                                counters.data_ptr())
        torch.cuda.synchronize()
        c = counters.cpu().numpy().astype(np.uint64)
        log(f"single-history launches: steps/launch {int(c[7])}")
        print(json.dumps({"mode": "single-history", "steps_per_launch": int(c[7]), "launches": 20}))
        return

    def make_req(engine):
        return pmc.Request(wl.n_histories, phases, request_id=wl.request_id, engine=engine,
                           block_size=a.block, chunk=a.chunk, refill_min=a.refill)

    ev_a = torch.cuda.Event(enable_timing=True)
    ev_b = torch.cuda.Event(enable_timing=True)

    def one_step(req, kernel_ms):
        for t in tallies:
            t.zero_()
        counters.zero_()
        ev_a.record(stream)
        pmc.pmc_dose_device(eng.ctx, req, stream.cuda_stream, [t.data_ptr() for t in tallies],
                            counters.data_ptr())
        ev_b.record(stream)
        for i, p in enumerate(phases):
            pmc.pmc_convert_device(eng.ctx, p, tallies[i].data_ptr(), wl.n_histories,
                                   stream.cuda_stream, doses[i].data_ptr(), None)
        kernel_ms.append((ev_a, ev_b))

    def run(engine, steps, warmup):
        req = make_req(engine)
        scratch = []
        for _ in range(warmup):
            one_step(req, scratch)
        torch.cuda.synchronize()
        spans = []
        ts = time.perf_counter()
        for _ in range(steps):
            k = []
            one_step(req, k)
            torch.cuda.synchronize()  # events are reused: read them per step
            spans.append(k[0][0].elapsed_time(k[0][1]))
        torch.cuda.synchronize()
        te = time.perf_counter()
        return req, (te - ts) / steps, spans

    def balance(req):
        c = counters.cpu().numpy().astype(np.uint64)
        dep = 0
        for t in tallies:
            lo = int((t & 0xFFFFFFFF).sum().item())
            hi = int((t >> 32).sum().item())
            dep += (hi << 32) + lo
        return pmc.pmc_balance_from_counters(eng.ctx, req, c, dep)

    log(f"batched engine: warmup {a.warmup}, steps {a.steps}")
    req_b, sec_b, spans_b = run(pmc.PMC_ENGINE_PERSISTENT, a.steps, a.warmup)
    bal = balance(req_b)
    assert bal["deposited"] + bal["escaped"] + bal["nuclear"] == bal["incident"], bal
    assert bal["histories"] == wl.n_histories
    steps_per_run = bal["steps"]
    kern_ms = float(np.mean(spans_b))
    log(f"batched: {sec_b * 1e3:.1f} ms/step, transport kernel {kern_ms:.1f} ms, "
        f"{steps_per_run / wl.n_histories:.1f} steps/history, balance exact")
    value = wl.n_histories / sec_b

    plain = None
    if not a.no_plain and a.plain_steps > 0:
        log(f"plain engine: steps {a.plain_steps}")
        req_p, sec_p, spans_p = run(pmc.PMC_ENGINE_PLAIN, a.plain_steps, 1)
        balp = balance(req_p)
        assert balp == bal, (balp, bal)  # same keys: the integer results are identical
        plain = {"value": wl.n_histories / sec_p, "ms_per_step": sec_p * 1e3,
                 "transport_ms": float(np.mean(spans_p)),
                 "speedup_batched_vs_plain": (wl.n_histories / sec_b) / (wl.n_histories / sec_p)}
        log(f"plain: {sec_p * 1e3:.1f} ms/step (x{plain['speedup_batched_vs_plain']:.2f} batched)")

    lane_steps_per_s = steps_per_run / (kern_ms * 1e-3)
    if VALU_PER_STEP:
        achieved = lane_steps_per_s * VALU_PER_STEP
        roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                    "unit": "T lane-VALU-instr/s", "frac": achieved / PEAK_LANE_OPS,
                    "traffic": None, "valu_per_step": VALU_PER_STEP,
                    "lane_steps_per_s": lane_steps_per_s, "kernel": "transport_persistent",
                    "kernel_ms": kern_ms}
    else:
        roofline = {"bound": "alu", "achieved": None, "peak": PEAK_LANE_OPS / 1e12,
                    "unit": "T lane-VALU-instr/s", "frac": None, "traffic": None,
                    "lane_steps_per_s": lane_steps_per_s, "kernel": "transport_persistent",
                    "kernel_ms": kern_ms}

    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baseline(wl, a.cpu_seconds)

    out = {
        "metric": "proton histories/s (batched 4D dose, one persistent launch over 10 phases)",
        "value": value, "unit": "histories/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": sec_b * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 transport, int64 tally",
        "data": "synthetic (seeded thorax phantom and plan; no patient data)",
        "config": {"workload": "thorax4d 10 phases x 256x256x160 @1.5x1.5x2 mm, 3000 spots, "
                               f"{wl.n_histories:.0e} histories",
                   "phases": len(phases), "grid": list(grid), "spots": int(len(wl.plan.spots)),
                   "histories": wl.n_histories, "steps_per_history": steps_per_run / wl.n_histories},
        "plain": plain,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    eng.close()


def cpu_baseline(wl, target_s):
    """The FP64 oracle on the host, on the first K histories of every spot."""
    import numpy as np
    import oracle
    oracle.build()
    cores = os.cpu_count() or 1
    k = 2
    t = time.perf_counter()
    _, b = oracle.dose_subset(wl.phases, wl.plan, wl.n_histories, wl.seed, 0, k, n_threads=cores)
    dt = time.perf_counter() - t
    k2 = max(k, int(k * target_s / max(dt, 1e-3)))
    k2 = min(k2, 4096)
    log(f"cpu baseline: calibration {b['histories']} histories in {dt:.2f} s; sample k={k2}/spot")
    t = time.perf_counter()
    _, b = oracle.dose_subset(wl.phases, wl.plan, wl.n_histories, wl.seed, 0, k2, n_threads=cores)
    dt = time.perf_counter() - t
    return {"value": b["histories"] / dt, "unit": "histories/s", "cores": cores, "kind": "oracle",
            "sample": f"first {k2} histories of every spot of the thorax4d plan "
                      f"({b['histories']} histories, {b['steps']} steps, {dt:.1f} s, FP64)",
            "steps_per_history": b["steps"] / max(b["histories"], 1)}


if __name__ == "__main__":
    main()
