"""Launch-shape autotuner for the persistent transport engine.

For a request shape (phase grids, number of phases and spots, history count
bucket, energy range) it times candidate launch shapes -- tally mode (lane or
block/core), threads per block, histories per work item and the lane-refill
threshold -- on a probe request over the same plan, and keeps the fastest.
Every candidate produces bit-identical tallies (integer fixed-point deposits,
histories keyed by (request, spot, history)), so the choice only affects
speed.  Choices are cached in a JSON file keyed by device and shape.

The probe should have the request's own history count where the block
engine is a candidate: its work items are runs of one spot's histories, so a
smaller probe has shorter items than the real request.
"""
from __future__ import annotations

import itertools
import json
import math
import os
import time
from typing import Dict, Optional, Sequence

from . import pmc

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "pmc", "autotune.json")

BLOCKS = (256, 512, 1024)
CHUNKS = (64, 256, 1024)
REFILLS = (32, 48, 64)
# (block, chunk, refill, tally mode)
LANE_CANDIDATES = [(b, c, r, pmc.PMC_TALLY_LANE) for b, c, r in itertools.product(BLOCKS, CHUNKS, REFILLS)]
CORE_CANDIDATES = [(1024, c, r, pmc.PMC_TALLY_CORE) for c in (4096, 8192, 16384) for r in (32, 64)]
# small requests: work items of a few histories per lane, so that every CU
# gets some
SMALL_CANDIDATES = (LANE_CANDIDATES
                    + [(1024, c, 64, pmc.PMC_TALLY_CORE) for c in (1024, 2048, 4096, 8192)])
# a short list for large requests, timed at full size
FULL_SIZE_CANDIDATES = CORE_CANDIDATES + [(1024, 256, 64, pmc.PMC_TALLY_LANE),
                                          (512, 64, 64, pmc.PMC_TALLY_LANE)]


def shape_key(device_name: str, grids: Sequence[Sequence[int]], n_spots: int, n_hist: int,
              e_range: Sequence[float], engine: int = pmc.PMC_ENGINE_PERSISTENT) -> str:
    g = "+".join("x".join(str(int(v)) for v in grid) for grid in grids)
    bucket = int(round(math.log10(max(n_hist, 1)) * 2))  # half-decade buckets
    return (f"{device_name}|engine{engine}|tally-modes|{len(grids)}ph|{g}|spots{n_spots}|h{bucket}|"
            f"E{e_range[0]:.0f}-{e_range[1]:.0f}")


def _load(path: str) -> Dict[str, dict]:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path: str, data: Dict[str, dict]) -> None:
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(ctx, phases: Sequence[int], key: str, dev_tallies: Sequence[int], dev_counters: int,
         stream: int, sync, probe_histories: int, request_id: int = 0, flags: int = 0,
         cache_path: Optional[str] = DEFAULT_CACHE, candidates=None, repeats: int = 2,
         log=None, prefer=None, tolerance: float = 0.01) -> dict:
    """Return {"block_size", "chunk", "refill_min", "tally_mode", "probe_ms"} for `key`.

    candidates: (block, chunk, refill[, tally mode]) tuples; the default is
    every lane-mode combination of BLOCKS x CHUNKS x REFILLS.

    prefer: a candidate (usually the library's own default shape) kept unless
    another one is faster by more than `tolerance`: shapes within the timing
    noise of each other would otherwise be picked at random from run to run.

    dev_tallies / dev_counters are caller-owned device buffers (they are
    overwritten by the probes; the engine adds into them, so the caller
    zeroes them before real use).  `sync` waits for `stream`.
    """
    cache = _load(cache_path) if cache_path else {}
    if key in cache:
        return cache[key]
    if candidates is None:
        candidates = LANE_CANDIDATES
    best = None
    preferred = None
    for cand in candidates:
        block, chunk, refill = cand[:3]
        mode = cand[3] if len(cand) > 3 else pmc.PMC_TALLY_LANE
        req = pmc.Request(probe_histories, phases, request_id=request_id, flags=flags,
                          engine=pmc.PMC_ENGINE_PERSISTENT, block_size=block, chunk=chunk,
                          refill_min=refill, tally_mode=mode)
        times = []
        for r in range(repeats + 1):
            sync()
            t0 = time.perf_counter()
            pmc.pmc_dose_device(ctx, req, stream, dev_tallies, dev_counters)
            sync()
            if r:  # the first run of a shape also rebuilds the request data
                times.append(time.perf_counter() - t0)
        ms = 1e3 * min(times)
        if log:
            log(f"autotune {block=} {chunk=} {refill=} {mode=}: {ms:.2f} ms")
        this = {"block_size": block, "chunk": chunk, "refill_min": refill, "tally_mode": mode,
                "probe_ms": ms, "probe_histories": probe_histories}
        if best is None or ms < best["probe_ms"]:
            best = this
        if prefer is not None and (block, chunk, refill, mode) == tuple(prefer):
            preferred = this
    if preferred is not None and preferred["probe_ms"] <= best["probe_ms"] * (1.0 + tolerance):
        best = preferred
    if cache_path:
        cache = _load(cache_path)
        cache[key] = best
        _store(cache_path, cache)
    return best
