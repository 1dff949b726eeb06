"""The no-allocation entry point, pmc_dose_device_noalloc, through the C ABI:
its tallies and counters equal pmc_dose_device's bit for bit (integer
results), over calls in a row on the library's one scratch array -- a large
request, then smaller ones, so that what the first left in the array must
not leak into the next -- for the block engine, the lane engine, the plain
engine, phases with different calibrations and FP64; it allocates no device
memory (the context's accounting does not move); a request too large for
the array is refused before any device work and leaves the outputs alone."""
import sys

import numpy as np
import pytest

from paper_1809_03927_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def run_both(torch, pmc, e, req, nvox):
    """(tallies, counters) of pmc_dose_device and of the no-allocation call."""
    st = torch.cuda.current_stream()
    out = []
    for noalloc in (False, True):
        tal = [torch.zeros(nvox, dtype=torch.int64, device="cuda") for _ in range(req.n_phases)]
        cnt = torch.zeros(pmc.PMC_COUNTERS, dtype=torch.int64, device="cuda")
        ptrs = [t.data_ptr() for t in tal]
        torch.cuda.synchronize()
        used = pmc.pmc_bytes_in_use(e.ctx)
        if noalloc:
            pmc.pmc_dose_device_noalloc(e.ctx, req, st.cuda_stream, ptrs, cnt.data_ptr())
            assert pmc.pmc_bytes_in_use(e.ctx) == used  # nothing allocated
        else:
            pmc.pmc_dose_device(e.ctx, req, st.cuda_stream, ptrs, cnt.data_ptr())
        torch.cuda.synchronize()
        out.append(([t.cpu().numpy() for t in tal], cnt.cpu().numpy()))
    return out


def check(torch, pmc, e, req, nvox, label):
    (ta, ca), (tb, cb) = run_both(torch, pmc, e, req, nvox)
    say(label, f"{int(ca[6])} histories, {int(ca[7])} steps")
    if req.c.item_end == 0:
        assert int(ca[6]) == req.c.n_histories
    else:
        assert 0 < int(ca[6]) < req.c.n_histories
    assert np.array_equal(ca, cb), label
    for i, (a, b) in enumerate(zip(ta, tb)):
        assert np.array_equal(a, b), (label, i)
    return ta


def test_noalloc_equals_dose_device():
    import torch
    from paper_1809_03927_amd import pmc
    wl = W.workload_thorax4d(n_histories=400_000, shape_xyz=(96, 96, 60))
    nvox = wl.phases[0].nvox
    e = pmc.Engine(device=0, seed=wl.seed)
    try:
        e.load_workload(wl)
        # a phase with another calibration: the request carries one LUT per phase
        e.load_phase(10, W.scaled_calibration(wl.phases[4], 1.035))
        plan = W.Plan(wl.plan.fields, wl.plan.spots.copy())
        plan.spots["phase"][plan.spots["phase"] == 4] = 10
        pmc.pmc_load_plan(e.ctx, 1, plan.fields, plan.spots)
        P = pmc.PMC_ENGINE_PERSISTENT
        cases = [
            ("10 phases, library's launch shape", pmc.Request(400_000, list(range(10)), engine=P)),
            ("block engine, 3 phases", pmc.Request(150_000, [0, 5, 9], engine=P, tally_mode=pmc.PMC_TALLY_CORE)),
            ("lane engine, 2 phases, small items", pmc.Request(60_000, [2, 7], engine=P,
                                                               tally_mode=pmc.PMC_TALLY_LANE, chunk=64)),
            ("plain engine, 1 phase", pmc.Request(20_000, [3], engine=pmc.PMC_ENGINE_PLAIN)),
            ("two calibrations (one LUT per phase)", pmc.Request(80_000, [3, 10], engine=P, plan=1)),
            ("a slice of the work items", pmc.Request(200_000, [0, 1], engine=P).slice(3, 40)),
        ]
        for label, req in cases:
            check(torch, pmc, e, req, nvox, label)
    finally:
        e.close()


def test_noalloc_fp64():
    import torch
    from paper_1809_03927_amd import pmc
    wl = W.workload_slabs()
    e = pmc.Engine(device=0, precision=pmc.PMC_FP64, seed=wl.seed)
    try:
        e.load_workload(wl)
        for n in (20_000, 3_000):
            check(torch, pmc, e, pmc.Request(n, [0], engine=pmc.PMC_ENGINE_PERSISTENT), wl.phases[0].nvox,
                  f"FP64 slabs {n}")
    finally:
        e.close()


def test_noalloc_refuses_requests_beyond_the_scratch():
    """100,000 spots need 12 MB of request data: PMC_E_RANGE, the tallies
    keep their contents and the next call works."""
    import torch
    from paper_1809_03927_amd import pmc
    ph = W.make_box((32, 32, 32), (2.5, 2.5, 2.5), 0, origin_mm=(-40.0, -40.0, 0.0))
    rows = [(100.0 + (i % 50), (i % 31) - 15.0, (i % 29) - 14.0, 4.0, 1.0, 0, 0) for i in range(100_000)]
    plan = W.Plan(W.plan_single().fields, W._spots(rows))
    e = pmc.Engine(device=0, seed=3)
    try:
        e.load_phase(0, ph)
        e.load_plan(plan)
        st = torch.cuda.current_stream()
        tal = torch.full((ph.nvox,), 77, dtype=torch.int64, device="cuda")
        cnt = torch.full((pmc.PMC_COUNTERS,), 5, dtype=torch.int64, device="cuda")
        req = pmc.Request(1_000_000, [0], engine=pmc.PMC_ENGINE_PERSISTENT)
        with pytest.raises(pmc.PmcError) as ex:
            pmc.pmc_dose_device_noalloc(e.ctx, req, st.cuda_stream, [tal.data_ptr()], cnt.data_ptr())
        assert ex.value.code == pmc.PMC_E_RANGE
        torch.cuda.synchronize()
        assert bool((tal == 77).all()) and bool((cnt == 5).all())
        small = W.Plan(plan.fields, plan.spots[:500].copy())
        e.load_plan(small)
        check(torch, pmc, e, pmc.Request(50_000, [0], engine=pmc.PMC_ENGINE_PERSISTENT), ph.nvox,
              "after a refused request")
    finally:
        e.close()
