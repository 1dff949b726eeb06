"""Benchmark of the proton dose engine on one MI355X.

One step = one full 4D dose calculation of the thorax workload (10 breathing
phases of 256x256x160 voxels, 3000 spots assigned to phases by the delivery
clock, 5e7 histories): zero the int64 tallies, transport all phases, convert
every phase's tally to dose.  Inputs (phantoms, tables, plan) are resident on
the device before timing.

Batched engine (the reported value): one persistent launch over a work queue
of all phases with an autotuned launch shape, the whole step captured in a
HIP graph and replayed.  Plain engine (reported beside it): one launch per
phase, one history per thread, no refill, no graph.  Both give identical
integer tallies (checked).

Also measured, each with its own check:
* roofline: the transport kernel's device-wide atomics against a replay of
  its own logged deposit addresses, and its VALU rate;
* serving: a Poisson stream of single-phase requests of mixed grid and
  history counts at loads 0.5, 0.8 and 1.2 x the plain engine's service
  rate, with the full and a forced 2 GiB device-memory budget; p50/p99 of
  arrival -> dose on the host against the plain engine run serially;
  identical doses per request;
* the 40^3 water and 128^3 slab configurations; phantoms shaped like the
  paper's lung, esophagus and liver cases (Table I grids); the robust-
  optimisation workload (90 calculations + influence matrices); delivery
  simulation, deformable accumulation and the 25-trial 4D loop;
* the FP64 oracle on the host (cpu_baseline), timed on a sample of the same
  histories and used as the accuracy check of the GPU's.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X: 256 CUs at 2.4 GHz; FP32 vector peak 157.3 TFLOP/s = 256 x 2.4e9 x
# 128 lanes x 2 flops (FMA), i.e. 128 lanes of ordinary (non-packed) VALU work
# per CU per clock: 7.86e13 lane operations per second.  (The counters agree:
# the block engine issues 1.09 wave64 VALU instructions per CU per clock, more
# than a 64-lane-per-clock CU could.)
PEAK_LANE_OPS = 256 * 128 * 2.4e9

# VALU instructions one lane executes per transport step of the FP32 kernel:
# SQ_INSTS_VALU of single-history launches (one active lane) divided by their
# step count (profiles/transport_valu_per_step_thorax.md).
VALU_PER_STEP = 448.6

# The method's own VALU work per step (one Philox4x32-10 block, two
# Box-Muller transforms, the table reads and the range inversion, the DDA),
# at the upper end of an estimate of 150-250 instructions per lane.
METHOD_VALU_PER_STEP = 250

# HBM-side bytes of one full-size transport launch (5e7 histories of the
# thorax 4D workload, block engine, chunk 8192), from FETCH_SIZE and
# WRITE_SIZE scaled by a 4 GiB copy calibration, and its memory-side atomic
# requests (TCC_EA0_ATOMIC_sum) (profiles/transport_core_thorax4d_counters.md).
# Valid only for the sources they were measured on (hash below) and that
# launch shape; otherwise null.
PROFILED_TRAFFIC_BYTES = 169.0e9
PROFILED_MEMSIDE_ATOMICS = 4.0190e9
# memory-side atomic requests of the replay probe per atomic it issues
# (TCC_EA0_ATOMIC_sum 2.1430e9 for 2.147e9 replayed, same profile)
PROFILED_REPLAY_MEMSIDE_PER_ISSUED = 2.1430e9 / 2.147e9
PROFILED_KERNEL_HASH = "a0dc63cd344b303c"

# Deformable accumulation (energy/mass transfer, Sec. 2.D.2): the per-phase
# tallies of the 4D run accumulated onto one reference phase with n^3
# subvoxels per voxel.  FP64 operations the plain definition spends on one
# subvoxel whose centre lies inside the DVF grid: centre 9 (3 x add, multiply,
# add), DVF grid coordinates 21 (3 subtractions, then per axis 3 multiplies,
# 2 adds, 1 divide), cell fractions 3, trilinear interpolation of the three
# translations 63 (7 lerps of 3 operations each) plus 3 adds, reference voxel
# 6 (3 subtractions, 3 divides).  Floors and comparisons are not counted.
ACC_REF_PHASE = 5
ACC_N_SUB = 5
ACC_OPS_PER_SUBVOXEL = 105
# Dose interpolation (Eq. (3)) per mapped subvoxel of a reference voxel: the
# same centre, grid coordinates, fractions and translation (99), then the
# dose sample: voxel-centre coordinates 9 (3 x subtract, divide, subtract),
# fractions 3, 7 lerps of 3 operations, and the add into the sum: 133.
DIM_OPS_PER_SUBVOXEL = 133
# These are unfused FP64 operations: one per lane per clock, 256 CUs x 64
# FP64 lanes x 2.4 GHz (the 78.6 TFLOP/s FP64 vector figure counts an FMA as
# two operations).
PEAK_FP64_OPS = 256 * 64 * 2.4e9
# HBM-side bytes of one accumulation call (9 sources of the thorax 4D
# workload onto phase 5, n_sub 5), FETCH_SIZE and WRITE_SIZE of emtm_push
# scaled like the transport's (profiles/emtm_push_thorax4d_counters.md);
# valid for the source it was measured on (hash of pmc_accumulate.hip).
PROFILED_ACC_TRAFFIC_BYTES = 3.13e9
PROFILED_DIM_TRAFFIC_BYTES = 4.40e9
PROFILED_ACC_HASH = "977f00a20898e340"

# Least pass fraction of the voxel criterion for a comparison with the oracle
# that shares its random numbers (FP32 and FP64 runs of the same histories).
SAME_SEED_MIN_PASS = 0.995


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
    p.add_argument("--no-tune", action="store_true", help="library default launch shape")
    p.add_argument("--tune-cache", type=str, default=None)
    p.add_argument("--no-graph", action="store_true")
    p.add_argument("--no-plain", action="store_true")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-atomic-probe", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--no-accumulation", action="store_true")
    p.add_argument("--no-delivery", action="store_true")
    p.add_argument("--no-fourd", action="store_true")
    p.add_argument("--fourd-trials", type=int, default=25)
    p.add_argument("--acc-cpu-seconds", type=float, default=10.0)
    p.add_argument("--latency-requests", type=int, default=200,
                   help="served-stream requests for the p50/p99 latency comparison (0 = skip)")
    p.add_argument("--latency-loads", type=str, default="0.5,0.8,1.2",
                   help="served-stream loads (x the plain engine's service rate)")
    p.add_argument("--latency-budgets-gb", type=str, default="0,2",
                   help="device-memory budgets of the serving loop, GiB (0 = 0.9 x free)")
    p.add_argument("--cases", type=str, default="lung,esophagus,liver",
                   help="patient-shaped 4D cases to measure ('' = none)")
    p.add_argument("--case-steps", type=int, default=3)
    p.add_argument("--case-cpu-seconds", type=float, default=5.0)
    p.add_argument("--no-robust", action="store_true")
    p.add_argument("--no-configs", action="store_true")
    p.add_argument("--mode", choices=["bench", "single-history", "copy-calibration", "accumulation-scan"],
                   default="bench")
    return p.parse_args()


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this engine runs on one GPU; sharding over several GPUs is a "
                                   "design note only", "n_gpus": a.gpus}))
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1809_03927_amd import autotune, pmc, serve
    from paper_1809_03927_amd import workloads as W

    served = None
    if a.mode == "bench" and a.latency_requests > 0:
        # phantoms of the served stream, generated in forked processes before
        # this process touches the GPU
        t0 = time.time()
        served = serve.prebuild(a.latency_requests, workers=8)
        log(f"served stream: {a.latency_requests} requests generated in {time.time() - t0:.1f} s")
    cases = {}
    if a.mode == "bench" and a.cases:
        for name in a.cases.split(","):
            t0 = time.time()
            cases[name] = W.workload_case(name, 50_000_000, workers=8)
            log(f"case {name}: {len(cases[name].plan.spots)} spots, 10 phases generated in {time.time() - t0:.1f} s")

    if a.mode == "copy-calibration":
        # plain device-to-device copies of 4 GiB (far larger than the 256 MB
        # last-level cache): the HBM counters of these dispatches calibrate
        # FETCH_SIZE / WRITE_SIZE (expected 4 GiB read and 4 GiB written each)
        n = 1 << 29
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "copy-calibration", "bytes_per_copy": n * 8, "copies": 3}))
        return

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
    tptr = [t.data_ptr() for t in tallies]

    if a.mode == "single-history":
        # one history per launch (one active lane): VALU instructions per step
        one = W.workload_thorax4d(1, shape_xyz=grid)
        one.plan.spots = one.plan.spots[:1].copy()
        one.plan.spots["phase"] = 0
        eng.load_plan(one.plan)
        req = pmc.Request(1, [0], engine=pmc.PMC_ENGINE_PLAIN, block_size=64)
        for _ in range(20):
            counters.zero_()
            pmc.pmc_dose_device(eng.ctx, req, stream.cuda_stream, [tptr[0]], counters.data_ptr())
        torch.cuda.synchronize()
        c = counters.cpu().numpy()
        print(json.dumps({"mode": "single-history", "steps_per_launch": int(c[7]), "launches": 20}))
        return

    if a.mode == "accumulation-scan":
        accumulation_scan(eng, wl, tallies, counters, stream, torch)
        return

    # ---- launch shape ----------------------------------------------------
    tuned = {"block_size": 0, "chunk": 0, "refill_min": 0, "tally_mode": 0}
    if not a.no_tune:
        e = wl.plan.spots["energy_MeV"]
        key = autotune.shape_key(torch.cuda.get_device_name(0), [grid] * len(phases),
                                 len(wl.plan.spots), wl.n_histories, (float(e.min()), float(e.max())))
        t1 = time.time()
        # full-size probes over a short candidate list (block-engine items are
        # runs of one spot's histories: a smaller probe would shorten them)
        dflt = pmc.pmc_launch_shape(eng.ctx, pmc.Request(wl.n_histories, phases, request_id=wl.request_id,
                                                         engine=pmc.PMC_ENGINE_PERSISTENT))
        tuned = autotune.tune(eng.ctx, phases, key, tptr, counters.data_ptr(), stream.cuda_stream,
                              torch.cuda.synchronize, wl.n_histories, request_id=wl.request_id,
                              cache_path=a.tune_cache or autotune.DEFAULT_CACHE,
                              candidates=autotune.FULL_SIZE_CANDIDATES, repeats=1,
                              prefer=(dflt["block_size"], dflt["chunk"], dflt["refill_min"], dflt["tally_mode"]))
        log(f"autotune ({time.time() - t1:.1f} s): tally mode {tuned['tally_mode']} block "
            f"{tuned['block_size']} chunk {tuned['chunk']} refill {tuned['refill_min']}")

    def make_req(engine):
        kw = {}
        if engine == pmc.PMC_ENGINE_PERSISTENT:
            kw = dict(block_size=tuned["block_size"], chunk=tuned["chunk"],
                      refill_min=tuned["refill_min"], tally_mode=tuned.get("tally_mode", 0))
        return pmc.Request(wl.n_histories, phases, request_id=wl.request_id, engine=engine, **kw)

    def eager_step(req):
        for t in tallies:
            t.zero_()
        counters.zero_()
        pmc.pmc_dose_device(eng.ctx, req, stream.cuda_stream, tptr, counters.data_ptr())
        for i, p in enumerate(phases):
            pmc.pmc_convert_device(eng.ctx, p, tptr[i], wl.n_histories, stream.cuda_stream,
                                   doses[i].data_ptr(), None)

    def balance(req):
        c = counters.cpu().numpy().astype(np.uint64)
        dep = 0
        for t in tallies:
            dep += (int((t >> 32).sum().item()) << 32) + int((t & 0xFFFFFFFF).sum().item())
        b = pmc.pmc_balance_from_counters(eng.ctx, req, c, dep)
        b["atomics"] = int(c[12])
        return b

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        ts = time.perf_counter()
        for e0, e1 in ev:
            e0.record(stream)
            fn()
            e1.record(stream)
        torch.cuda.synchronize()
        te = time.perf_counter()
        return (te - ts) / steps, [e0.elapsed_time(e1) for e0, e1 in ev]

    # ---- batched engine: graph replay of the whole step --------------------
    req_b = make_req(pmc.PMC_ENGINE_PERSISTENT)
    graph = None
    if not a.no_graph:
        eager_step(req_b)  # builds the request data once
        torch.cuda.synchronize()
        graph = pmc.pmc_graph_create(eng.ctx, req_b, tptr, counters.data_ptr(),
                                     [d.data_ptr() for d in doses])
        step_b = lambda: pmc.pmc_graph_launch(graph, stream.cuda_stream, eng.ctx)
    else:
        step_b = lambda: eager_step(req_b)
    log(f"batched engine ({'graph' if graph else 'eager'}): warmup {a.warmup}, steps {a.steps}")
    sec_b, spans_b = timed(step_b, a.steps, a.warmup)
    bal = balance(req_b)
    assert bal["deposited"] + bal["escaped"] + bal["nuclear"] == bal["incident"], bal
    assert bal["histories"] == wl.n_histories
    tal_b = [t.clone() for t in tallies]
    log(f"batched: {sec_b * 1e3:.1f} ms/step (GPU {np.mean(spans_b):.1f} ms), "
        f"{bal['steps'] / wl.n_histories:.1f} steps/history, balance exact")

    # transport kernel alone, same launch shape, timed with events on its stream
    def transport_only():
        pmc.pmc_dose_device(eng.ctx, req_b, stream.cuda_stream, tptr, counters.data_ptr())
    _, spans_k = timed(transport_only, max(2, min(a.steps, 3)), 0)
    kern_ms = float(np.mean(spans_k))

    delivery = None
    if not a.no_delivery:
        delivery = delivery_bench(eng, None if a.no_cpu_baseline else 2)

    accumulation = None
    if not a.no_accumulation:
        accumulation = accumulation_bench(eng, wl, tal_b, stream, timed, max(2, min(a.steps, 5)),
                                          None if a.no_cpu_baseline else a.acc_cpu_seconds)
    fourd_out = None
    if not a.no_fourd and a.fourd_trials > 0:
        fourd_out = fourd_bench(eng, wl, a.fourd_trials, tuned.get("tally_mode", 0))
    shape_b = pmc.pmc_launch_shape(eng.ctx, req_b)
    kernel_name = ("transport_core<float>" if shape_b["tally_mode"] == pmc.PMC_TALLY_CORE
                   else "transport_persistent<float>")

    plain = None
    if not a.no_plain and a.plain_steps > 0:
        req_p = make_req(pmc.PMC_ENGINE_PLAIN)
        log(f"plain engine: steps {a.plain_steps}")
        sec_p, spans_p = timed(lambda: eager_step(req_p), a.plain_steps, 1)
        balp = balance(req_p)
        same = all(torch.equal(x, y) for x, y in zip(tal_b, tallies))
        assert same and balp["deposited"] == bal["deposited"], "plain and batched tallies differ"
        plain = {"value": wl.n_histories / sec_p, "ms_per_step": sec_p * 1e3,
                 "speedup_batched_vs_plain": sec_p / sec_b, "tallies_identical": same}
        log(f"plain: {sec_p * 1e3:.1f} ms/step -> batched is x{sec_p / sec_b:.3f}")

    probe = None
    if not a.no_atomic_probe and shape_b["tally_mode"] == pmc.PMC_TALLY_CORE:
        probe = atomic_probe(eng, pmc, wl, phases, tuned, tallies, counters, stream, torch)
        log(f"atomic replay of the kernel's own addresses: {probe['per_s'] / 1e9:.2f} G/s "
            f"({probe['replayed']:.3g} atomics in {probe['ms']:.1f} ms)")
    roofline = roofline_fields(bal, kern_ms, probe, kernel_name, shape_b, wl, grid, pmc)
    if graph is not None:
        pmc.pmc_graph_destroy(graph)
        graph = True
    # the GPU's share of the accuracy check: the histories the oracle sample
    # runs (the first k of every spot = the first round of work items of k)
    gpu_sample = None
    k_sample = None
    if not a.no_cpu_baseline:
        k_sample = cpu_sample_size(wl, a.cpu_seconds)
        per = pmc.pmc_split_histories(wl.plan.spots, phases, wl.n_histories)
        req_s = pmc.Request(wl.n_histories, phases, request_id=wl.request_id,
                            engine=pmc.PMC_ENGINE_PERSISTENT, chunk=k_sample,
                            tally_mode=tuned.get("tally_mode", 0), item_begin=0,
                            item_end=int(np.count_nonzero(per)))
        for t in tallies:
            t.zero_()
        pmc.pmc_dose_device(eng.ctx, req_s, stream.cuda_stream, tptr, counters.data_ptr())
        torch.cuda.synchronize()
        gpu_sample = [t.cpu().numpy() for t in tallies]
    eng.close()
    latency = None
    serving = None
    if served is not None:
        loads = [float(x) for x in a.latency_loads.split(",")]
        budgets = [int(float(x) * 2**30) for x in a.latency_budgets_gb.split(",")]
        log(f"served stream: {a.latency_requests} requests at loads {loads}, budgets {a.latency_budgets_gb} GiB "
            f"(0 = 0.9 x free)")
        res = serve.run_grid(a.latency_requests, loads, budgets, prebuilt=served,
                             log=lambda m: log("serve:", m))
        keys = ("p50_latency_s", "p99_latency_s", "mean_latency_s", "max_latency_s",
                "throughput_hist_per_s", "makespan_s", "slices", "peak_bytes", "phantom_loads", "evictions")
        workload = (f"served stream: {a.latency_requests} single-phase thorax requests, grids 64^3 to "
                    f"256x256x160, 50-3000 spots, 1e5-5e7 histories (log-uniform), Poisson arrivals at a "
                    f"load x the plain engine's service rate")
        serving = {"workload": workload, "plain_calibration_hist_per_s": res["plain_calibration_hist_per_s"],
                   "scenarios": [{"load": sc["load"], "budget": sc["budget"], "budget_bytes": sc["budget_bytes"],
                                  "arrival_rate_hz": sc["arrival_rate_hz"],
                                  "batched": {k: sc["batched"].get(k) for k in keys},
                                  "plain_serial": {k: sc["plain_serial"].get(k) for k in keys},
                                  "identical_doses": sc["identical_doses"],
                                  "batched_p99_le_plain": sc["batched"]["p99_latency_s"]
                                  <= sc["plain_serial"]["p99_latency_s"]}
                                 for sc in res["scenarios"]]}
        head = next((sc for sc in serving["scenarios"] if sc["load"] == 0.8 and sc["budget"] == "full"),
                    serving["scenarios"][0])
        latency = {"workload": workload.replace("a load", f"{head['load']}"), "load": head["load"],
                   "budget": head["budget"], "arrival_rate_hz": head["arrival_rate_hz"],
                   "batched": head["batched"], "plain_serial": head["plain_serial"],
                   "identical_doses": head["identical_doses"], "requests": a.latency_requests}
        for sc in serving["scenarios"]:
            log(f"latency load {sc['load']} budget {sc['budget']}: batched p50/p99 "
                f"{sc['batched']['p50_latency_s'] * 1e3:.0f}/{sc['batched']['p99_latency_s'] * 1e3:.0f} ms, "
                f"plain {sc['plain_serial']['p50_latency_s'] * 1e3:.0f}/"
                f"{sc['plain_serial']['p99_latency_s'] * 1e3:.0f} ms, identical {sc['identical_doses']}")
    configs = None if a.no_configs else configs_bench(not a.no_cpu_baseline)
    case_out = {}
    for name, cwl in cases.items():
        case_out[name] = case_bench(cwl, a.case_steps, 1, 0 if a.no_cpu_baseline else a.case_cpu_seconds)
        cases[name] = None
    robust_out = None if a.no_robust else robust_bench(0 if a.no_cpu_baseline else 5.0)
    cpu = None if a.no_cpu_baseline else cpu_baseline(wl, k_sample, gpu_sample, single_thread=True)
    out = {
        "metric": "proton histories/s; p50/p99 dose-request latency, batched vs plain, 1 MI355X",
        "value": wl.n_histories / sec_b, "unit": "histories/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": sec_b * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 transport, int64 tally",
        "data": "synthetic (seeded thorax phantom and plan; no patient data)",
        "config": {"workload": f"thorax4d: 10 phases x {grid[0]}x{grid[1]}x{grid[2]} @1.5x1.5x2 mm, "
                               f"3000 spots, {wl.n_histories:.0e} histories",
                   "phases": len(phases), "grid": list(grid), "spots": int(len(wl.plan.spots)),
                   "histories": wl.n_histories, "steps_per_history": bal["steps"] / wl.n_histories,
                   "launch": tuned, "graph": graph is not None},
        "plain": plain,
        "latency": latency,
        "serving": serving,
        "cases": case_out or None,
        "robust": robust_out,
        "configs": configs,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "accumulation": accumulation,
        "delivery": delivery,
        "fourd": fourd_out,
    }
    print(json.dumps(out))


def source_hash(files):
    """Hash of the code of the given sources: comments removed and white
    space collapsed, so that a profile stays valid across edits of comments
    alone (the sources hold no comment markers inside string literals)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1809_03927_amd", "csrc", f), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
        h.update(b"\0")
    return h.hexdigest()[:16]


def kernel_hash():
    return source_hash(("pmc_device.hpp", "pmc_kernels.hip", "pmc_host.cpp"))


LOG_PER_LANE = 8192  # logged atomics per lane of the replay probe


def atomic_probe(eng, pmc, wl, phases, tuned, tallies, counters, stream, torch):
    """The device-wide atomic throughput of the transport kernel's own
    deposit-address pattern: one block-engine launch of the benchmark's
    request (same shape, one block per CU) logs the address of every lane's
    device-wide tally atomic (the first LOG_PER_LANE of each lane), then a
    replay kernel issues exactly those atomics, per lane in logged order,
    back to back; timed with events on the benchmark's stream.  Leaves the
    tallies changed (run after every use of them)."""
    import numpy as np
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    req = pmc.Request(wl.n_histories, phases, request_id=wl.request_id, engine=pmc.PMC_ENGINE_PERSISTENT,
                      chunk=tuned["chunk"], refill_min=tuned["refill_min"], tally_mode=pmc.PMC_TALLY_CORE,
                      grid_blocks=n_cu)
    lanes = n_cu * 1024
    log_buf = torch.empty(LOG_PER_LANE * lanes, dtype=torch.int64, device="cuda")
    count = torch.zeros(lanes, dtype=torch.int32, device="cuda")
    for t in tallies:
        t.zero_()
    counters.zero_()
    pmc.pmc_atomic_log(eng.ctx, req, stream.cuda_stream, [t.data_ptr() for t in tallies], counters.data_ptr(),
                       log_buf.data_ptr(), LOG_PER_LANE, count.data_ptr())
    torch.cuda.synchronize()
    c = count.cpu().numpy().astype(np.int64)
    replayed = int(np.minimum(c, LOG_PER_LANE).sum())
    spans = []
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        pmc.pmc_atomic_replay(eng.ctx, stream.cuda_stream, log_buf.data_ptr(), LOG_PER_LANE,
                              count.data_ptr(), lanes)
        e1.record(stream)
        torch.cuda.synchronize()
        spans.append(e0.elapsed_time(e1))
    del log_buf
    torch.cuda.empty_cache()
    ms = float(np.mean(spans[1:]))
    return {"per_s": replayed / (ms * 1e-3), "ms": ms, "replayed": replayed, "lanes": lanes,
            "logged_total": int(c.sum()), "per_lane_cap": LOG_PER_LANE}


def roofline_fields(bal, kern_ms, probe, kernel_name, shape_b, wl, grid, pmc):
    """The dominant kernel's roofline: device-wide int64 atomics per second
    against the replay of its own address pattern (the binding roof of the
    block engine), with the VALU view beside it.  Rates are memory-side
    requests (TCC_EA0_ATOMIC_sum of the profile of these sources, over the
    live-timed durations) when the profile matches the sources and launch;
    else the atomics each kernel issues (exact counts, live)."""
    kern_s = kern_ms * 1e-3
    issued = bal["atomics"] / kern_s
    lane_steps_s = bal["steps"] / kern_s
    default_cfg = wl.n_histories == 50_000_000 and grid == (256, 256, 160)
    profiled = (default_cfg and kernel_hash() == PROFILED_KERNEL_HASH
                and shape_b["tally_mode"] == pmc.PMC_TALLY_CORE and shape_b["chunk"] == 8192)
    out = {"kernel": kernel_name, "kernel_ms": kern_ms, "atomics_per_launch": int(bal["atomics"]),
           "traffic": PROFILED_TRAFFIC_BYTES if profiled else None,
           "traffic_unit": "HBM bytes per launch (FETCH_SIZE x 2.0 + WRITE_SIZE, rocprofv3, copy-calibrated)"}
    if probe:
        replay_s = probe["ms"] * 1e-3
        issued_peak = probe["per_s"]
        if profiled:
            achieved = PROFILED_MEMSIDE_ATOMICS / kern_s
            peak = probe["replayed"] * PROFILED_REPLAY_MEMSIDE_PER_ISSUED / replay_s
            unit = "G memory-side int64 atomics/s"
        else:
            achieved, peak, unit = issued, issued_peak, "G device-wide int64 atomics/s (issued)"
        out.update({
            "bound": "atomic", "achieved": achieved / 1e9, "peak": peak / 1e9, "unit": unit,
            "frac": achieved / peak,
            "memory_side_atomics_per_launch": PROFILED_MEMSIDE_ATOMICS if profiled else None,
            "issued": {"achieved": issued / 1e9, "peak": issued_peak / 1e9, "frac": issued / issued_peak},
            "peak_source": (f"pmc_atomic_replay of the kernel's logged deposit addresses: the first "
                            f"{probe['per_lane_cap']} device-wide atomics of each of its {probe['lanes']} lanes "
                            f"({probe['replayed']:.4g} of {probe['logged_total']:.4g}), in logged order, back "
                            f"to back, {probe['ms']:.1f} ms"),
        })
    else:
        out.update({"bound": "alu", "achieved": lane_steps_s * VALU_PER_STEP / 1e12,
                    "peak": PEAK_LANE_OPS / 1e12, "unit": "T lane-VALU-instr/s",
                    "frac": lane_steps_s * VALU_PER_STEP / PEAK_LANE_OPS})
    out["valu"] = {
        "peak_T_lane_instr_per_s": PEAK_LANE_OPS / 1e12,
        "lane_steps_per_s": lane_steps_s,
        "executed_per_step": VALU_PER_STEP,
        "frac_executed": lane_steps_s * VALU_PER_STEP / PEAK_LANE_OPS,
        "method_per_step": METHOD_VALU_PER_STEP,
        "frac_method": lane_steps_s * METHOD_VALU_PER_STEP / PEAK_LANE_OPS,
    }
    return out


SCAN_N = (1, 2, 3, 4, 5, 6, 8, 10, 16)


def accumulation_scan(eng, wl, tallies, counters, stream, torch):
    """Accumulation time and tumour dose-volume histograms against the
    voxel-subdivision scale n for both methods (the studies of the paper's
    Figs. 3 and 4, on the synthetic thorax): one 4D transport of the
    workload, then the nine other phases accumulated onto phase 5 with
    EMTM and DIM for each n; DVHs of the phase-5 tumour compared with n = 16."""
    import numpy as np
    from paper_1809_03927_amd import fourd, pmc
    from paper_1809_03927_amd import workloads as W
    phases = list(range(len(wl.phases)))
    req = pmc.Request(wl.n_histories, phases, request_id=wl.request_id, engine=pmc.PMC_ENGINE_PERSISTENT)
    pmc.pmc_dose_device(eng.ctx, req, stream.cuda_stream, [t.data_ptr() for t in tallies], counters.data_ptr())
    torch.cuda.synchronize()
    ref = ACC_REF_PHASE
    src = [p for p in phases if p != ref]
    for p in src:
        pmc.pmc_load_dvf(eng.ctx, 100 + p, W.thorax_dvf(p, ref, n_phases=len(phases)))
        pmc.pmc_load_dvf(eng.ctx, 300 + p, W.thorax_dvf(ref, p, n_phases=len(phases)))
    nv = wl.phases[ref].nvox
    dose = torch.empty(nv, dtype=torch.float64, device="cuda")
    roi = W.thorax_tumour_mask(tuple(wl.phases[ref].shape_xyz), ref, len(phases)).ravel()
    out = {"mode": "accumulation-scan", "workload": f"thorax4d ({wl.n_histories:.0e} histories), phases {src} "
                                                     f"onto phase {ref}; ROI: the phase-{ref} tumour "
                                                     f"({int(roi.sum())} voxels)", "methods": {}}
    for method, fn, base in (("emtm", pmc.pmc_accumulate_device, 100), ("dim", pmc.pmc_accumulate_dim_device, 300)):
        rows, doses = [], {}
        for n in SCAN_N:
            def run():
                fn(eng.ctx, ref, tallies[ref].data_ptr(), src, [base + p for p in src],
                   [tallies[p].data_ptr() for p in src], n, wl.n_histories, stream.cuda_stream,
                   dose.data_ptr(), None)
            run()
            torch.cuda.synchronize()
            reps = 2 if n <= 10 else 1
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                run()
            e1.record(stream)
            torch.cuda.synchronize()
            doses[n] = dose.cpu().numpy()
            rows.append({"n": n, "ms": e0.elapsed_time(e1) / reps})
            log(f"scan {method} n={n}: {rows[-1]['ms']:.2f} ms")
        top = doses[SCAN_N[-1]][roi]
        bins = np.linspace(0.0, 1.1 * float(top.max()), 221)
        dvh_ref = fourd.dvh(doses[SCAN_N[-1]], roi, bins)
        for r in rows:
            d = doses[r["n"]][roi]
            r["dvh_max_diff"] = float(np.max(np.abs(fourd.dvh(doses[r["n"]], roi, bins) - dvh_ref)))
            r["d95_rel"] = float(np.percentile(d, 5) / np.percentile(top, 5))
            r["d50_rel"] = float(np.median(d) / np.median(top))
        out["methods"][method] = rows
    print(json.dumps(out))


def fourd_bench(eng, wl, trials, tally_mode):
    """The whole 4D dose calculation (fourd.FourD), trial by trial, on the
    thorax 4D workload: the delivery-uncertainty study of Sec. 2.B (start
    phase, period U{3..7} s with sigma 0.4 s, synchrotron parameters;
    repainted at 0.005 MU as the paper's clinical plans), sub-plans per
    phase, the Monte Carlo of all ten phases in one batched launch
    (wl.n_histories per trial), EMTM accumulation onto phase 5 with n = 5.
    Wall time per component, as the paper's Table II."""
    import numpy as np
    from paper_1809_03927_amd import fourd, pmc
    from paper_1809_03927_amd import workloads as W
    ref = ACC_REF_PHASE
    ids = list(range(len(wl.phases)))
    dvf_ids = [None] * len(ids)
    for p in ids:
        if p != ref:
            pmc.pmc_load_dvf(eng.ctx, 500 + p, W.thorax_dvf(p, ref, n_phases=len(ids)))
            dvf_ids[p] = 500 + p
    sp = wl.plan.spots.copy()
    sp["weight"] = sp["weight"] / sp["weight"].sum() * 250.0
    fd = fourd.FourD(eng.ctx, wl.plan.fields, sp, ids, ref, dvf_ids, wl.phases[0].nvox, n_sub=ACC_N_SUB,
                     tally_mode=tally_mode)
    d = W.Delivery(n_trials=trials, period_sd_s=0.4, period_min_s=3, period_max_s=7, max_mu=0.005, seed=31)
    fd.run(W.Delivery(**{**d.__dict__, "n_trials": 1}), wl.n_histories, keep=False)  # warm-up
    t0 = time.perf_counter()
    out = fd.run(d, wl.n_histories, request_id=1000, keep=False)
    total = time.perf_counter() - t0
    fd.close()
    mc = float(np.mean(out["time_mc_s"]))
    acc = float(np.mean(out["time_accumulation_s"]))
    host = float(np.mean(out["time_host_s"]))
    dl = out["time_delivery_s"] / trials
    log(f"4D dose: {trials} trials in {total:.2f} s: per trial delivery {dl * 1e3:.1f} ms (one call for all), "
        f"device MC {mc * 1e3:.0f} ms, accumulation {acc * 1e3:.0f} ms; host load + enqueue {host * 1e3:.0f} ms "
        f"(overlapped with the previous trial)")
    return {
        "workload": f"thorax4d phases and plan (250 MU, {len(sp)} spots), {trials} delivery trials "
                    f"(start phase U{{0..9}}, period U{{3..7}} s, sigma 0.4 s, synchrotron uncertainty, "
                    f"repainted 0.005 MU), {wl.n_histories:.0e} histories per 4D dose, EMTM n={ACC_N_SUB} "
                    f"onto phase {ref}",
        "trials": trials, "total_s": total, "s_per_trial": total / trials,
        "per_trial_s": {"delivery": dl, "mc_device": mc, "accumulation_device": acc,
                        "host_load_and_enqueue": host},
        "mean_delivery_time_s": float(out["delivery"]["time"].mean()),
        "context": "the paper's Table II: 246-367 s per 4D dose (delivery 7 s, MC 135-175 s on eight GTX "
                   "Titan X, accumulation 45-122 s); other hardware and inputs",
    }


DELIVERY_TRIALS = 25
DELIVERY_SCALING_TRIALS = (25, 100, 400)
DELIVERY_SCENARIOS = {
    "free": {},
    "gated": {"gate_lo": 3, "gate_hi": 7},        # CT30-CT70, 50 % duty cycle
    "repainted": {"max_mu": 0.005},               # isolayered, 0.005 MU per delivery
}


def delivery_bench(eng, cpu_trials):
    """The paper's delivery-uncertainty study (Sec. 2.B): 25 trials of the
    3-field robust plan with random start phase, breathing period U{3..7} s
    (sigma 0.4 s) and synchrotron uncertainty, free-breathing, gated and
    repainted; each call simulates all trials and fields (one GPU thread per
    trial and field) and returns the MU per spot and phase.  Timed as whole
    calls (inputs and outputs in host memory).  Then the oracle replays the
    first trials of the repainted scenario, timed, and must match the GPU:
    MU and fills identical, end times within 1e-12, per timeline."""
    import numpy as np
    from paper_1809_03927_amd import pmc
    from paper_1809_03927_amd import workloads as W
    plan = W.plan_robust()
    sp = plan.spots.copy()
    sp["weight"] = sp["weight"] / sp["weight"].sum() * 600.0  # 600 MU over the three fields
    n_f = len(plan.fields)
    out = {"workload": f"robust plan: {n_f} fields, {len(sp)} spots, 600 MU; {DELIVERY_TRIALS} trials "
                       "(start phase U{0..9}, period U{3..7} s with sigma 0.4 s, synchrotron uncertainty); "
                       "synthetic synchrotron timing",
           "unit": "spot deliveries simulated/s", "scenarios": {}}
    results = {}
    for name, kw in DELIVERY_SCENARIOS.items():
        d = W.Delivery(n_trials=DELIVERY_TRIALS, period_sd_s=0.4, period_min_s=3, period_max_s=7, seed=17, **kw)
        pmc.pmc_delivery_simulate(eng.ctx, d, sp, n_f)  # warm-up
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            res = pmc.pmc_delivery_simulate(eng.ctx, d, sp, n_f)
        sec = (time.perf_counter() - t0) / reps
        n_del = int(np.count_nonzero(res["mu"]))  # (spot, phase) cells reached; deliveries below
        if d.max_mu > 0:
            pieces = np.ceil(sp["weight"] / d.max_mu)
            deliveries = float(pieces.sum()) * DELIVERY_TRIALS
        else:
            deliveries = float(len(sp)) * DELIVERY_TRIALS
        results[name] = (d, res)
        out["scenarios"][name] = {
            "ms_per_call": sec * 1e3, "deliveries": deliveries, "value": deliveries / sec,
            "delivery_time_s_mean": float(res["time"].mean()), "fills_mean": float(res["fills"].mean()),
            "phase_cells_with_mu": n_del}
        log(f"delivery {name}: {sec * 1e3:.1f} ms per call of {DELIVERY_TRIALS} trials x {n_f} fields "
            f"({deliveries:.3g} deliveries), mean delivery time {res['time'].mean():.0f} s")
    rp = out["scenarios"]["repainted"]
    out["value"] = rp["value"]
    out["ms_per_call"] = rp["ms_per_call"]
    # scaling with the number of trials (repainted): every (trial, field)
    # timeline is one block, so throughput grows with the timelines until
    # they fill the device; the MU output (trials x spots x 10 doubles)
    # comes back to the host in each call
    d0 = results["repainted"][0]
    scaling = []
    for n_t in DELIVERY_SCALING_TRIALS:
        d = W.Delivery(**{**d0.__dict__, "n_trials": n_t})
        pmc.pmc_delivery_simulate(eng.ctx, d, sp, n_f)
        t0 = time.perf_counter()
        pmc.pmc_delivery_simulate(eng.ctx, d, sp, n_f)
        sec = time.perf_counter() - t0
        deliveries = float(np.ceil(sp["weight"] / d.max_mu).sum()) * n_t
        scaling.append({"trials": n_t, "timelines": n_t * n_f, "ms_per_call": sec * 1e3,
                        "deliveries_per_s": deliveries / sec})
        log(f"delivery scaling: {n_t} trials ({n_t * n_f} timelines) {sec * 1e3:.1f} ms, "
            f"{deliveries / sec:.3g} deliveries/s")
    out["trial_scaling"] = scaling
    out["roofline"] = {
        "bound": "latency",
        "note": "each (trial, field) timeline is serial: 75 threads, one dependent FP64 chain each; "
                "the figure is deliveries per second per timeline",
        "achieved": rp["value"] / (DELIVERY_TRIALS * n_f), "unit": "deliveries/s per timeline",
        "peak": None, "frac": None, "traffic": None}
    if cpu_trials:
        import oracle.delivery as DL
        d, res = results["repainted"]
        d1 = W.Delivery(**{**d.__dict__, "n_trials": cpu_trials})
        t0 = time.perf_counter()
        want = DL.simulate(sp, n_f, d1)
        dt = time.perf_counter() - t0
        deliveries = float(np.ceil(sp["weight"] / d.max_mu).sum()) * cpu_trials
        # per (trial, field): MU per (spot, phase) and fills identical, end
        # time within 1e-12; a timeline that differs must hold a decision at
        # a near tie in the oracle's log (the Box-Muller logarithm and cosine
        # of host and device may differ in the last bit)
        identical, flipped, bad, t_rel = 0, 0, 0, 0.0
        for f in range(n_f):
            idx = np.flatnonzero(sp["field"] == f)
            for t in range(cpu_trials):
                if (np.array_equal(want["mu"][t, idx], res["mu"][t, idx])
                        and want["fills"][t, f] == res["fills"][t, f]):
                    identical += 1
                    t_rel = max(t_rel, abs(res["time"][t, f] - want["time"][t, f]) / max(want["time"][t, f], 1.0))
                elif want["margin"][t, f] < 1e-10:
                    flipped += 1
                else:
                    bad += 1
        ok = bad == 0 and flipped <= 1 and t_rel <= 1e-12
        out["cpu_baseline"] = {"value": deliveries / dt, "unit": "spot deliveries simulated/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"the first {cpu_trials} trials of the repainted scenario "
                                         f"({deliveries:.3g} deliveries) in {dt:.1f} s, pure Python",
                               "accuracy": {"check": "GPU vs oracle per (trial, field) timeline: MU per spot and "
                                                     "phase and fills identical, end time within 1e-12 relative, "
                                                     "or a logged near-tie decision (at most one timeline)",
                                            "timelines_identical": identical, "timelines_flipped_at_tie": flipped,
                                            "end_time_max_rel": t_rel, "passed": bool(ok)}}
        log(f"delivery oracle: {cpu_trials} trials in {dt:.1f} s; {identical} timelines identical, "
            f"{flipped} flipped at a near tie, {bad} differing, end time max rel {t_rel:.1e}")
    return out


def mapped_subvoxels(ph, dvf, n, with_mass=True):
    """Subvoxel centres of the phase's voxels (with mass, if with_mass) that
    lie inside the grid box of an axis-aligned DVF (the subvoxels that are
    mapped)."""
    import numpy as np
    assert tuple(dvf.row) == (1.0, 0.0, 0.0) and tuple(dvf.col) == (0.0, 1.0, 0.0)
    nz, ny, nx = ph.hu.shape
    cnt = []
    for axis, m in enumerate((nx, ny, nz)):
        c = (np.arange(m)[:, None] + (np.arange(n)[None, :] + 0.5) / n) * ph.spacing_mm[axis]
        g = (ph.origin_mm[axis] + c - dvf.start_mm[axis]) / dvf.spacing_mm[axis]
        cnt.append(((g >= 0.0) & (g <= dvf.n[axis] - 1)).sum(axis=1).astype(np.float64))
    hu = np.clip(ph.hu, -1024, 3071).astype(np.float64)
    has_mass = np.interp(hu, np.asarray(ph.calib_hu, float), np.asarray(ph.calib_rho, float)) > 0
    if ph.mask is not None:
        has_mass &= ph.mask.astype(bool)
    if not with_mass:
        has_mass = np.ones(ph.hu.shape, dtype=bool)
    return float(np.einsum("zyx,x,y,z->", has_mass.astype(np.float64), cnt[0], cnt[1], cnt[2]))


def accumulation_bench(eng, wl, tallies, stream, timed, steps, cpu_seconds):
    """All other phases' tallies accumulated onto the reference phase by
    energy/mass transfer (pmc_accumulate_device on the stream the events are
    recorded on), with the FP64-operation roofline; then the oracle on a
    z-slab of one source phase, timed, and the GPU's result for the same
    slab checked against it."""
    import numpy as np
    import torch
    from paper_1809_03927_amd import pmc
    from paper_1809_03927_amd import workloads as W
    ref = ACC_REF_PHASE
    n = ACC_N_SUB
    src = [p for p in range(len(wl.phases)) if p != ref]
    t0 = time.time()
    dvfs = {p: W.thorax_dvf(p, ref, n_phases=len(wl.phases)) for p in src}
    for p in src:
        pmc.pmc_load_dvf(eng.ctx, 100 + p, dvfs[p])
    log(f"accumulation: {len(src)} DVFs {dvfs[src[0]].n} built and loaded in {time.time() - t0:.1f} s")
    nv = wl.phases[ref].nvox
    dose = torch.empty(nv, dtype=torch.float64, device="cuda")
    mask = torch.empty(nv, dtype=torch.uint8, device="cuda")

    def run():
        pmc.pmc_accumulate_device(eng.ctx, ref, tallies[ref].data_ptr(), src, [100 + p for p in src],
                                  [tallies[p].data_ptr() for p in src], n, wl.n_histories,
                                  stream.cuda_stream, dose.data_ptr(), mask.data_ptr())
    _, spans = timed(run, steps, 1)
    ms = float(np.mean(spans))
    mapped = sum(mapped_subvoxels(wl.phases[p], dvfs[p], n) for p in src)
    achieved = ACC_OPS_PER_SUBVOXEL * mapped / (ms * 1e-3)
    default_size = wl.phases[ref].hu.shape == (160, 256, 256) and len(wl.phases) == 10
    log(f"accumulation: {ms:.2f} ms for {len(src)} source phases (n_sub {n}), "
        f"{mapped / (ms * 1e-3) / 1e9:.1f} G subvoxels/s")
    out = {
        "workload": f"EMTM: phases {src} of the thorax4d run accumulated onto phase {ref}, n_sub {n}, "
                    f"DVFs {dvfs[src[0]].n[0]}x{dvfs[src[0]].n[1]}x{dvfs[src[0]].n[2]} @2.5 mm",
        "value": mapped / (ms * 1e-3), "unit": "mapped subvoxels/s", "ms_per_accumulation": ms,
        "ms_per_source_phase": ms / len(src), "mapped_subvoxels": mapped, "dtype": "f64 mapping, int64 sums",
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_OPS / 1e12,
                     "unit": "T FP64 op/s (unfused)", "frac": achieved / PEAK_FP64_OPS,
                     "traffic": (PROFILED_ACC_TRAFFIC_BYTES if default_size and
                                 source_hash(["pmc_accumulate.hip"]) == PROFILED_ACC_HASH else None),
                     "traffic_unit": "bytes per accumulation call (HBM side)",
                     "ops_per_subvoxel": ACC_OPS_PER_SUBVOXEL,
                     "kernel": "emtm_push (with the reference dose, per-source fill and ratio, mask)"},
        "cpu_baseline": None,
    }
    if cpu_seconds:
        out["cpu_baseline"] = accumulation_cpu(eng, wl, tallies, dvfs, src[0], ref, n, cpu_seconds)
    out["dim"] = dim_bench(eng, wl, tallies, stream, timed, steps, cpu_seconds)
    return out


def dim_bench(eng, wl, tallies, stream, timed, steps, cpu_seconds):
    """The same accumulation by dose interpolation (pmc_accumulate_dim_device:
    reference-to-source DVFs, one thread per reference voxel), with its
    FP64-operation roofline; then the oracle's Eq. (3) on a z-slab of the
    reference phase, timed, and the GPU's result for that slab checked
    against it."""
    import numpy as np
    import torch
    from paper_1809_03927_amd import pmc
    from paper_1809_03927_amd import workloads as W
    ref = ACC_REF_PHASE
    n = ACC_N_SUB
    src = [p for p in range(len(wl.phases)) if p != ref]
    dvfs = {p: W.thorax_dvf(ref, p, n_phases=len(wl.phases)) for p in src}
    for p in src:
        pmc.pmc_load_dvf(eng.ctx, 300 + p, dvfs[p])
    nv = wl.phases[ref].nvox
    dose = torch.empty(nv, dtype=torch.float64, device="cuda")
    mask = torch.empty(nv, dtype=torch.uint8, device="cuda")

    def run():
        pmc.pmc_accumulate_dim_device(eng.ctx, ref, tallies[ref].data_ptr(), src, [300 + p for p in src],
                                      [tallies[p].data_ptr() for p in src], n, wl.n_histories,
                                      stream.cuda_stream, dose.data_ptr(), mask.data_ptr())
    _, spans = timed(run, steps, 1)
    ms = float(np.mean(spans))
    mapped = sum(mapped_subvoxels(wl.phases[ref], dvfs[p], n, with_mass=False) for p in src)
    achieved = DIM_OPS_PER_SUBVOXEL * mapped / (ms * 1e-3)
    log(f"dose interpolation: {ms:.2f} ms for {len(src)} source phases (n_sub {n}), "
        f"{mapped / (ms * 1e-3) / 1e9:.1f} G subvoxels/s")
    out = {
        "workload": f"DIM: phases {src} of the thorax4d run pulled onto phase {ref}, n_sub {n}, "
                    f"reference-to-source DVFs {dvfs[src[0]].n[0]}x{dvfs[src[0]].n[1]}x{dvfs[src[0]].n[2]} "
                    f"@2.5 mm",
        "value": mapped / (ms * 1e-3), "unit": "mapped subvoxels/s", "ms_per_accumulation": ms,
        "ms_per_source_phase": ms / len(src), "mapped_subvoxels": mapped, "dtype": "f64",
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_OPS / 1e12,
                     "unit": "T FP64 op/s (unfused)", "frac": achieved / PEAK_FP64_OPS,
                     "traffic": (PROFILED_DIM_TRAFFIC_BYTES if wl.phases[ref].hu.shape == (160, 256, 256)
                                 and len(wl.phases) == 10
                                 and source_hash(["pmc_accumulate.hip"]) == PROFILED_ACC_HASH else None),
                     "traffic_unit": "bytes per accumulation call (HBM side)",
                     "ops_per_subvoxel": DIM_OPS_PER_SUBVOXEL,
                     "kernel": "dim_pull (with the source and reference doses, mask)"},
        "cpu_baseline": None,
    }
    if cpu_seconds:
        out["cpu_baseline"] = dim_cpu(eng, wl, tallies, dvfs, src[0], ref, n, cpu_seconds)
    return out


def dim_cpu(eng, wl, tallies, dvfs, sp, ref, n, target_s):
    """The oracle's Eq. (3) for a z-slab of the reference phase (through the
    middle of the grid) from source phase sp, timed; then the GPU's pull onto
    the same slab (as a phase of its own, zero reference tally) against it:
    masks identical, doses within 1e-12 relative.  The source tally is a
    seeded synthetic one (workloads.random_tally), not the run's: no input of
    the comparison comes from the library."""
    import dataclasses
    import numpy as np
    import torch
    import oracle
    import oracle.dim as D
    import oracle.emtm as E
    from paper_1809_03927_amd import pmc
    rph, sph, dvf = wl.phases[ref], wl.phases[sp], dvfs[sp]
    nz = rph.hu.shape[0]
    from paper_1809_03927_amd import workloads as W
    t_src = W.random_tally(sph, 11)
    rho_s = oracle.convert(sph, np.zeros(sph.hu.size, dtype=np.int64), 1)[1]
    dose_s = E.phase_dose(t_src, rho_s, float(np.prod(np.asarray(sph.spacing_mm) * 0.1)), wl.n_histories)

    def slab(k):
        z0 = nz // 2 - k // 2
        o = (rph.origin_mm[0], rph.origin_mm[1], rph.origin_mm[2] + z0 * rph.spacing_mm[2])
        return dataclasses.replace(rph, hu=np.ascontiguousarray(rph.hu[z0:z0 + k]), origin_mm=o, mask=None)

    def pull(k):
        c = slab(k)
        t1 = time.perf_counter()
        d = D.pull(c, sph, dose_s, dvf, n)
        return c, d, time.perf_counter() - t1

    _, _, dt1 = pull(1)
    k = int(min(nz, max(1, target_s / max(dt1, 1e-3))))
    c, term, dt = pull(k)
    mapped = mapped_subvoxels(c, dvf, n, with_mass=False)
    want_mask = E.report_mask(c, [dvf])
    want = np.where(want_mask, term, 0.0)
    out = {"value": mapped / dt, "unit": "mapped subvoxels/s", "cores": 1, "kind": "oracle",
           "sample": f"{k} z-slices of phase {ref} ({c.hu.size} voxels, {mapped:.3g} mapped subvoxels, "
                     f"n_sub {n}) pulled from phase {sp} by the numpy oracle in {dt:.1f} s"}
    pmc.pmc_load_phase(eng.ctx, 201, c)
    zero = torch.zeros(c.hu.size, dtype=torch.int64, device="cuda")
    dose = torch.empty(c.hu.size, dtype=torch.float64, device="cuda")
    mask = torch.empty(c.hu.size, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    ts = torch.from_numpy(t_src).cuda()
    torch.cuda.synchronize()
    pmc.pmc_accumulate_dim_device(eng.ctx, 201, zero.data_ptr(), [sp], [300 + sp], [ts.data_ptr()], n,
                                  wl.n_histories, 0, dose.data_ptr(), mask.data_ptr())
    torch.cuda.synchronize()
    pmc.pmc_unload_phase(eng.ctx, 201)
    got, gmask = dose.cpu().numpy(), mask.cpu().numpy().astype(bool)
    sel = want > 0
    rel = float(np.max(np.abs(got[sel] - want[sel]) / want[sel])) if sel.any() else 0.0
    same_mask = bool(np.array_equal(gmask, want_mask))
    out["accuracy"] = {"check": "GPU vs oracle on the sample: report masks identical, doses within 1e-12 "
                                "relative", "voxels": int(sel.sum()), "max_rel": rel,
                       "bit_identical_frac": float(np.mean(got == want)),
                       "passed": bool(same_mask and rel <= 1e-12 and sel.any())}
    log(f"dose interpolation oracle: {k} slices in {dt:.1f} s; GPU check max rel {rel:.2e}, "
        f"mask identical {same_mask}")
    return out


def accumulation_cpu(eng, wl, tallies, dvfs, sp, ref, n, target_s):
    """The oracle's energy/mass push of a z-slab of source phase sp (through
    the middle of the grid) onto the reference, timed; then the GPU's
    accumulation of the same slab (as a phase of its own, with a zero
    reference tally) against it: masks identical, doses within 1e-9.  The
    slab's tally is a seeded synthetic one (workloads.random_tally), not the
    run's: no input of the comparison comes from the library."""
    import dataclasses
    import numpy as np
    import torch
    import oracle
    import oracle.emtm as E
    from paper_1809_03927_amd import pmc
    ph, rph, dvf = wl.phases[sp], wl.phases[ref], dvfs[sp]
    nz = ph.hu.shape[0]
    from paper_1809_03927_amd import workloads as W
    tal = W.random_tally(ph, 7).reshape(ph.hu.shape)

    def slab(k):
        z0 = nz // 2 - k // 2
        o = (ph.origin_mm[0], ph.origin_mm[1], ph.origin_mm[2] + z0 * ph.spacing_mm[2])
        c = dataclasses.replace(ph, hu=np.ascontiguousarray(ph.hu[z0:z0 + k]), origin_mm=o,
                                mask=None if ph.mask is None else np.ascontiguousarray(ph.mask[z0:z0 + k]))
        return c, np.ascontiguousarray(tal[z0:z0 + k]).ravel()

    def push(k):
        c, t = slab(k)
        rho = oracle.convert(c, np.zeros(c.hu.size, dtype=np.int64), 1)[1]
        t1 = time.perf_counter()
        sums = E.push(c, t, rho, rph, dvf, n)
        return c, t, sums, time.perf_counter() - t1

    _, _, _, dt1 = push(1)
    k = int(min(nz, max(1, target_s / max(dt1, 1e-3))))
    c, t, sums, dt = push(k)
    mapped = mapped_subvoxels(c, dvf, n)
    v_src = float(np.prod(np.asarray(c.spacing_mm) * 0.1))
    want_mask = E.report_mask(rph, [dvf])
    want = np.where(want_mask, E.dose_from_sums(sums, v_src, wl.n_histories), 0.0)
    out = {"value": mapped / dt, "unit": "mapped subvoxels/s", "cores": 1, "kind": "oracle",
           "sample": f"{k} z-slices of phase {sp} ({c.hu.size} voxels, {mapped:.3g} mapped subvoxels, "
                     f"n_sub {n}) pushed onto phase {ref} by the numpy oracle in {dt:.1f} s"}
    pmc.pmc_load_phase(eng.ctx, 200, c)
    zero = torch.zeros(rph.nvox, dtype=torch.int64, device="cuda")
    ts = torch.from_numpy(t).cuda()
    dose = torch.empty(rph.nvox, dtype=torch.float64, device="cuda")
    mask = torch.empty(rph.nvox, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    pmc.pmc_accumulate_device(eng.ctx, ref, zero.data_ptr(), [200], [100 + sp], [ts.data_ptr()], n,
                              wl.n_histories, 0, dose.data_ptr(), mask.data_ptr())
    torch.cuda.synchronize()
    pmc.pmc_unload_phase(eng.ctx, 200)
    got, gmask = dose.cpu().numpy(), mask.cpu().numpy().astype(bool)
    sel = want > 0
    rel = float(np.max(np.abs(got[sel] - want[sel]) / want[sel])) if sel.any() else 0.0
    same_mask = bool(np.array_equal(gmask, want_mask))
    out["accuracy"] = {"check": "GPU vs oracle on the sample: report masks identical, doses within 1e-9 "
                                "relative (identical binning of every subvoxel)",
                       "voxels": int(sel.sum()), "max_rel": rel,
                       "bit_identical_frac": float(np.mean(got == want)),
                       "passed": bool(same_mask and np.allclose(got, want, rtol=1e-9, atol=0) and sel.any())}
    log(f"accumulation oracle: {k} slices in {dt:.1f} s; GPU check max rel {rel:.2e}, "
        f"mask identical {same_mask}")
    return out


def cpu_sample_size(wl, target_s):
    """Histories per spot (first k of every spot) for about target_s seconds
    of the FP64 oracle on this host."""
    import oracle
    oracle.build()
    k = 2
    t = time.perf_counter()
    _, b = oracle.dose_subset(wl.phases, wl.plan, wl.n_histories, wl.seed, 0, k,
                              n_threads=os.cpu_count() or 1)
    dt = time.perf_counter() - t
    k2 = min(4096, max(k, int(k * target_s / max(dt, 1e-3))))
    log(f"cpu baseline: calibration {b['histories']} histories in {dt:.2f} s; sample k={k2}/spot")
    return k2


def cpu_baseline(wl, k, gpu_sample, label=None, single_thread=False):
    """The FP64 oracle on the host, on the first k histories of every spot,
    timed (with single_thread also on one thread, on the first k / cores
    histories of every spot); then the accuracy check of the GPU's tallies
    of the same histories against it: voxels above 10 % of the phase's
    maximum dose pass if |dD| <= 1 % of that maximum or <= 3 sigma_diff
    (sqrt 2 x the oracle's sigma from 10 history batches), in at least 99.5 %
    of them (the same random numbers); total energy within 0.1 %."""
    import numpy as np
    import oracle
    cores = os.cpu_count() or 1
    t = time.perf_counter()
    _, b = oracle.dose_subset(wl.phases, wl.plan, wl.n_histories, wl.seed, 0, k, n_threads=cores,
                              request_id=wl.request_id)
    dt = time.perf_counter() - t
    out = {"value": b["histories"] / dt, "unit": "histories/s", "cores": cores, "kind": "oracle",
           "sample": f"first {k} histories of every spot of the {label or wl.name} plan "
                     f"({b['histories']} histories, {b['steps']} steps, {dt:.1f} s, FP64)",
           "steps_per_history": b["steps"] / max(b["histories"], 1)}
    if single_thread:
        k1 = max(1, k // cores)
        t = time.perf_counter()
        _, b1 = oracle.dose_subset(wl.phases, wl.plan, wl.n_histories, wl.seed, 0, k1, n_threads=1,
                                   request_id=wl.request_id)
        dt1 = time.perf_counter() - t
        out["threads_1"] = {"value": b1["histories"] / dt1, "histories": b1["histories"], "seconds": dt1,
                            "sample": f"first {k1} histories of every spot"}
        log(f"cpu baseline on one thread: {b1['histories']} histories in {dt1:.1f} s "
            f"({b1['histories'] / dt1:.3g} histories/s)")
    if gpu_sample is None:
        return out
    nb = 10
    s1 = [np.zeros(ph.hu.size) for ph in wl.phases]
    s2 = [np.zeros(ph.hu.size) for ph in wl.phases]
    for r in range(nb):
        tb, _ = oracle.dose_subset(wl.phases, wl.plan, wl.n_histories, wl.seed, 0, k, n_threads=cores,
                                   request_id=wl.request_id, h_mod=nb, h_rem=r)
        for i, x in enumerate(tb):
            x = x.astype(np.float64)
            s1[i] += x
            s2[i] += x * x
    n_sel = n_ok = 0
    e_gpu = e_orc = 0.0
    for i, ph in enumerate(wl.phases):
        _, rho = oracle.convert(ph, np.zeros(ph.hu.size, dtype=np.int64), 1)
        inv = np.where(rho > 0, 1.0 / np.where(rho > 0, rho, 1.0), 0.0)
        mean_b = s1[i] / nb
        var_b = np.maximum((s2[i] - nb * mean_b * mean_b) / (nb - 1), 0.0)
        d_o = s1[i] * inv
        d_g = gpu_sample[i].astype(np.float64) * inv
        sig = np.sqrt(2.0 * nb * var_b) * inv
        dmax = d_o.max()
        if dmax > 0:
            sel = d_o > 0.1 * dmax
            dd = np.abs(d_g[sel] - d_o[sel])
            n_sel += int(sel.sum())
            n_ok += int(((dd <= 0.01 * dmax) | (dd <= 3.0 * sig[sel])).sum())
        e_gpu += float(gpu_sample[i].sum(dtype=np.float64))
        e_orc += float(s1[i].sum())
    frac = n_ok / max(n_sel, 1)
    e_rel = abs(e_gpu - e_orc) / max(e_orc, 1)
    out["accuracy"] = {"check": "GPU (FP32, same histories and random numbers) vs oracle (FP64) on the sample: "
                                "voxels above 10 % of the phase maximum within 1 % of it or 3 sigma_diff in at "
                                "least 99.5 % of them; total energy within 0.1 %",
                       "voxels": n_sel, "pass_frac": frac, "energy_rel": e_rel,
                       "passed": bool(frac >= SAME_SEED_MIN_PASS and e_rel <= 1e-3)}
    log(f"accuracy on the {label or wl.name} sample: {n_sel} voxels above 10 % Dmax, pass {frac:.4f}, "
        f"dE {e_rel:.2e}")
    return out


def gpu_first_k(eng, pmc, wl, phases, k, tally_mode, tallies, counters, stream, torch):
    """The GPU's tallies of the first k histories of every spot of the
    request: the first round of work items of k histories (queue order:
    the first run of every spot, in plan order)."""
    import numpy as np
    per = pmc.pmc_split_histories(wl.plan.spots, phases, wl.n_histories)
    req = pmc.Request(wl.n_histories, phases, request_id=wl.request_id, engine=pmc.PMC_ENGINE_PERSISTENT,
                      chunk=k, tally_mode=tally_mode, item_begin=0, item_end=int(np.count_nonzero(per)))
    for t in tallies:
        t.zero_()
    pmc.pmc_dose_device(eng.ctx, req, stream.cuda_stream, [t.data_ptr() for t in tallies], counters.data_ptr())
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in tallies]


def case_bench(wl, steps, plain_steps, cpu_seconds):
    """One 4D dose calculation of a patient-shaped case (10 phases, the
    case's plan, wl.n_histories): the library's default launch shape and
    its graph, timed as the thorax step; the plain engine beside it
    (identical tallies); the oracle on a sample of the same histories."""
    import numpy as np
    import torch
    from paper_1809_03927_amd import pmc
    eng = pmc.Engine(device=0, precision=pmc.PMC_FP32, seed=wl.seed)
    try:
        eng.load_workload(wl)
        phases = list(range(len(wl.phases)))
        nv = wl.phases[0].nvox
        tallies = [torch.zeros(nv, dtype=torch.int64, device="cuda") for _ in phases]
        doses = [torch.zeros(nv, dtype=torch.float64, device="cuda") for _ in phases]
        counters = torch.zeros(pmc.PMC_COUNTERS, dtype=torch.int64, device="cuda")
        stream = torch.cuda.current_stream()
        tptr = [t.data_ptr() for t in tallies]
        req_b = pmc.Request(wl.n_histories, phases, request_id=wl.request_id, engine=pmc.PMC_ENGINE_PERSISTENT)
        shape = pmc.pmc_launch_shape(eng.ctx, req_b)

        def eager(req):
            for t in tallies:
                t.zero_()
            counters.zero_()
            pmc.pmc_dose_device(eng.ctx, req, stream.cuda_stream, tptr, counters.data_ptr())
            for i, p in enumerate(phases):
                pmc.pmc_convert_device(eng.ctx, p, tptr[i], wl.n_histories, stream.cuda_stream,
                                       doses[i].data_ptr(), None)

        def timed(fn, n, warm):
            for _ in range(warm):
                fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(n):
                fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) / n

        def balance(req):
            c = counters.cpu().numpy().astype(np.uint64)
            dep = sum((int((t >> 32).sum().item()) << 32) + int((t & 0xFFFFFFFF).sum().item()) for t in tallies)
            b = pmc.pmc_balance_from_counters(eng.ctx, req, c, dep)
            b["atomics"] = int(c[12])
            return b

        eager(req_b)
        torch.cuda.synchronize()
        g = pmc.pmc_graph_create(eng.ctx, req_b, tptr, counters.data_ptr(), [d.data_ptr() for d in doses])
        try:
            sec_b = timed(lambda: pmc.pmc_graph_launch(g, stream.cuda_stream, eng.ctx), steps, 1)
        finally:
            pmc.pmc_graph_destroy(g)
        bal = balance(req_b)
        assert bal["deposited"] + bal["escaped"] + bal["nuclear"] == bal["incident"], bal
        assert bal["histories"] == wl.n_histories
        tal_b = [t.clone() for t in tallies]
        req_p = pmc.Request(wl.n_histories, phases, request_id=wl.request_id, engine=pmc.PMC_ENGINE_PLAIN)
        sec_p = timed(lambda: eager(req_p), plain_steps, 0)
        same = all(torch.equal(x, y) for x, y in zip(tal_b, tallies))
        assert same, f"{wl.name}: plain and batched tallies differ"
        del tal_b
        c = wl.name.split("4d_")[0]
        out = {"workload": f"{c}-shaped 4D: 10 phases x {'x'.join(map(str, wl.phases[0].shape_xyz))} at "
                           f"{'x'.join(f'{v:g}' for v in wl.phases[0].spacing_mm)} mm, {len(wl.plan.spots)} spots "
                           f"in {len(wl.plan.fields)} fields, {wl.n_histories:.0e} histories",
               "value": wl.n_histories / sec_b, "unit": "histories/s", "ms_per_step": sec_b * 1e3,
               "steps": steps, "steps_per_history": bal["steps"] / wl.n_histories,
               "atomics_per_history": bal["atomics"] / wl.n_histories,
               "spots_per_phase": np.bincount(wl.plan.spots["phase"], minlength=len(phases)).tolist(),
               "launch": {k: shape[k] for k in ("block_size", "chunk", "refill_min", "tally_mode")},
               "plain": {"value": wl.n_histories / sec_p, "ms_per_step": sec_p * 1e3,
                         "speedup_batched_vs_plain": sec_p / sec_b, "tallies_identical": same}}
        log(f"{c}: batched {sec_b * 1e3:.1f} ms/step ({wl.n_histories / sec_b:.3g} histories/s, "
            f"{bal['steps'] / wl.n_histories:.1f} steps/history), plain {sec_p * 1e3:.1f} ms (x{sec_p / sec_b:.2f})")
        if cpu_seconds:
            k = cpu_sample_size(wl, cpu_seconds)
            sample = gpu_first_k(eng, pmc, wl, phases, k, shape["tally_mode"], tallies, counters, stream, torch)
            out["cpu_baseline"] = cpu_baseline(wl, k, sample, label=c)
        return out
    finally:
        eng.close()


def robust_bench(cpu_seconds):
    """Robust-optimisation scale (the future use of Sec. 4.C): the thorax 4D
    phantom, 10 phases x 9 scenarios of the 3-field 8000-spot plan, 2e7
    histories per calculation, all 90 arriving at once, through the serving
    loop (batched) and one after the other with the plain engine (doses
    identical); the 1 % influence matrix of the nominal scenario on all ten
    phases.  The oracle checks a sample of one calculation (RSP x 1.035,
    phase 3)."""
    import numpy as np
    import torch
    from paper_1809_03927_amd import pmc, robust
    from paper_1809_03927_amd import workloads as W
    res = robust.run(n_histories=20_000_000, log=lambda m: log("robust:", m))
    keys = ("p50_latency_s", "p99_latency_s", "mean_latency_s", "max_latency_s", "throughput_hist_per_s",
            "makespan_s")
    out = {"workload": f"robust: thorax 4D 10 phases x 9 scenarios (setup +-3 mm x/y/z, RSP x 1.035/0.965) "
                       f"= {res['calculations']} calculations of the 3-field {res['spots']}-spot plan, "
                       f"{res['histories_per_calculation']:.0e} histories each, all arriving at once",
           "value": res["batched"]["throughput_hist_per_s"], "unit": "histories/s",
           "batched": {k: res["batched"][k] for k in keys},
           "plain_serial": {k: res["plain-serial"][k] for k in keys},
           "speedup_batched_vs_plain": res["plain-serial"]["makespan_s"] / res["batched"]["makespan_s"],
           "identical_doses": res["identical_doses"], "calculations": res["calculations"],
           "influence": {k: res["influence"][k] for k in ("rel_threshold", "total_seconds", "total_nnz",
                                                          "histories_per_s")}}
    out["influence"]["per_phase_ms"] = [round(x["seconds"] * 1e3, 1) for x in res["influence"]["phases"]]
    log(f"robust: batched {res['batched']['makespan_s']:.2f} s, plain {res['plain-serial']['makespan_s']:.2f} s "
        f"(x{out['speedup_batched_vs_plain']:.2f}); influence {res['influence']['total_seconds']:.2f} s for 10 phases")
    if cpu_seconds:
        name, shift, scale = W.ROBUST_SCENARIOS[7]
        ph = W.scaled_calibration(W.make_thorax((256, 256, 160), 3, 10), scale)
        plan = W.plan_robust(5, shift_mm=shift)
        plan.spots["phase"] = 0
        wl = W.Workload(f"robust_{name}_phase3", [ph], plan, 20_000_000, seed=5)
        eng = pmc.Engine(device=0, precision=pmc.PMC_FP32, seed=wl.seed)
        try:
            eng.load_workload(wl)
            tallies = [torch.zeros(ph.nvox, dtype=torch.int64, device="cuda")]
            counters = torch.zeros(pmc.PMC_COUNTERS, dtype=torch.int64, device="cuda")
            k = cpu_sample_size(wl, cpu_seconds)
            sample = gpu_first_k(eng, pmc, wl, [0], k, 0, tallies, counters, torch.cuda.current_stream(), torch)
        finally:
            eng.close()
        out["cpu_baseline"] = cpu_baseline(wl, k, sample, label=f"robust {name} phase 3")
    return out


def configs_bench(cpu):
    """The two single-phase configurations: 40^3 water with one 150 MeV spot
    (1e5 histories) and the 128^3 slabs with 500 spots (1e7 histories):
    histories/s of the persistent engine (autotuned over lane and block
    shapes, items of a few histories per lane included) and of the plain
    engine; the oracle timed at one thread and at every host thread (the
    water case in full, the slabs on the first 20 and 200 histories of every
    spot)."""
    import numpy as np
    import torch
    from paper_1809_03927_amd import autotune, pmc
    from paper_1809_03927_amd import workloads as W
    out = {}
    for wl in (W.workload_tiny(), W.workload_slabs()):
        eng = pmc.Engine(device=0, precision=pmc.PMC_FP32, seed=wl.seed)
        try:
            eng.load_workload(wl)
            nv = wl.phases[0].nvox
            t = torch.zeros(nv, dtype=torch.int64, device="cuda")
            c = torch.zeros(pmc.PMC_COUNTERS, dtype=torch.int64, device="cuda")
            st = torch.cuda.current_stream()
            res = {}
            e = wl.plan.spots["energy_MeV"]
            key = autotune.shape_key(torch.cuda.get_device_name(0), [wl.phases[0].shape_xyz],
                                     len(wl.plan.spots), wl.n_histories, (float(e.min()), float(e.max())))
            dflt = pmc.pmc_launch_shape(eng.ctx, pmc.Request(wl.n_histories, [0], request_id=wl.request_id,
                                                             engine=pmc.PMC_ENGINE_PERSISTENT))
            tuned = autotune.tune(eng.ctx, [0], key, [t.data_ptr()], c.data_ptr(), st.cuda_stream,
                                  torch.cuda.synchronize, wl.n_histories, request_id=wl.request_id,
                                  cache_path=None, candidates=autotune.SMALL_CANDIDATES, repeats=2,
                                  prefer=(dflt["block_size"], dflt["chunk"], dflt["refill_min"], dflt["tally_mode"]))
            shape = {k: tuned[k] for k in ("block_size", "chunk", "refill_min", "tally_mode")}
            for label, engine in (("batched", pmc.PMC_ENGINE_PERSISTENT), ("plain", pmc.PMC_ENGINE_PLAIN)):
                kw = shape if engine == pmc.PMC_ENGINE_PERSISTENT else {}
                req = pmc.Request(wl.n_histories, [0], request_id=wl.request_id, engine=engine, **kw)
                spans = []
                for r in range(4):
                    t.zero_()
                    c.zero_()
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record(st)
                    pmc.pmc_dose_device(eng.ctx, req, st.cuda_stream, [t.data_ptr()], c.data_ptr())
                    e1.record(st)
                    torch.cuda.synchronize()
                    if r:
                        spans.append(e0.elapsed_time(e1))
                res[label] = {"value": wl.n_histories / (np.mean(spans) * 1e-3), "ms": float(np.mean(spans))}
                res[label + "_tally"] = t.clone()
            same = torch.equal(res.pop("batched_tally"), res.pop("plain_tally"))
        finally:
            eng.close()
        entry = {"workload": wl.name, "histories": wl.n_histories, "unit": "histories/s",
                 "batched": {**res["batched"], "launch": shape}, "plain": res["plain"],
                 "speedup_batched_vs_plain": res["batched"]["value"] / res["plain"]["value"],
                 "tallies_identical": bool(same)}
        if cpu:
            import oracle
            cores = os.cpu_count() or 1
            k1, kn = (None, None) if wl.n_histories <= 100_000 else (20, 200)
            orc = {}
            for threads, k in ((1, k1), (cores, kn)):
                t0 = time.perf_counter()
                if k is None:
                    _, _, b = oracle.dose(wl.phases, wl.plan, wl.n_histories, wl.seed, n_threads=threads,
                                          with_dose=False)
                else:
                    _, b = oracle.dose_subset(wl.phases, wl.plan, wl.n_histories, wl.seed, 0, k, n_threads=threads)
                dt = time.perf_counter() - t0
                orc[f"threads_{threads}"] = {"value": b["histories"] / dt, "histories": b["histories"],
                                             "seconds": dt, "full_run": k is None}
            entry["cpu_baseline"] = {"kind": "oracle", "unit": "histories/s", "cores": cores, **orc}
        log(f"{wl.name}: batched {entry['batched']['value']:.3g}, plain {entry['plain']['value']:.3g} histories/s"
            + (f"; oracle {entry['cpu_baseline']}" if cpu else ""))
        out[wl.name] = entry
    return out


if __name__ == "__main__":
    main()
