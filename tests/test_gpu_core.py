"""Block engine (PMC_TALLY_CORE) on the GPU, through the C ABI: deposits
accumulated per spot in LDS and flushed once per work item give integer
tallies identical to the plain engine's, for every work-item size, phase
count and slicing, for beams along a grid axis (box-shaped cores) and
oblique to it (slice cores that follow the beam)."""
import sys

import numpy as np
import pytest

from paper_1809_03927_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def P():
    from paper_1809_03927_amd import pmc
    return pmc


def engine(P, wl):
    e = P.Engine(device=0, precision=P.PMC_FP32, seed=wl.seed)
    e.load_workload(wl)
    return e


def thorax_phase(shape, n):
    ph = W.make_thorax(shape, 0, 10)
    plan = W.plan_thorax(3, n_phases=10)
    plan.spots["phase"] = 0
    return W.Workload("thorax_phase", [ph], plan, n, seed=3)


def test_core_mode_equals_plain(P):
    wl = W.workload_slabs()
    n = 200_000
    e = engine(P, wl)
    try:
        say("core vs plain, slabs", n)
        _, t_plain, _, b_plain = e.dose(n, [0], engine=P.PMC_ENGINE_PLAIN)
        for launch in [dict(), dict(chunk=100), dict(chunk=5000, refill_min=1),
                       dict(chunk=777, refill_min=33, grid_blocks=7)]:
            say("core", launch)
            req = P.Request(n, [0], engine=P.PMC_ENGINE_PERSISTENT, tally_mode=P.PMC_TALLY_CORE, **launch)
            shape = P.pmc_launch_shape(e.ctx, req)
            assert shape["tally_mode"] == P.PMC_TALLY_CORE and shape["block_size"] == 1024
            assert shape["core_capacity"] > 0
            _, t_c, _, b_c = e.dose(n, [0], engine=P.PMC_ENGINE_PERSISTENT,
                                    tally_mode=P.PMC_TALLY_CORE, **launch)
            assert np.array_equal(t_c[0], t_plain[0]), launch
            assert b_c == b_plain
    finally:
        e.close()


@pytest.mark.parametrize("shape", [(64, 64, 40), (128, 128, 80)])
def test_core_mode_thorax_windows(P, shape):
    """At 128x128x80 the spot boxes exceed the LDS capacity (a window of the
    box is the core); at 64x64x40 they fit whole."""
    wl = thorax_phase(shape, 300_000)
    e = engine(P, wl)
    try:
        say("core vs plain, thorax phase", shape)
        _, t_plain, _, b_plain = e.dose(wl.n_histories, [0], engine=P.PMC_ENGINE_PLAIN)
        for chunk in (0, 64):
            _, t_c, _, b_c = e.dose(wl.n_histories, [0], engine=P.PMC_ENGINE_PERSISTENT,
                                    tally_mode=P.PMC_TALLY_CORE, chunk=chunk)
            assert np.array_equal(t_c[0], t_plain[0]), chunk
            assert b_c == b_plain
        boxes = P.pmc_influence_boxes(e.ctx, 0, 0, len(wl.plan.spots))
        cap = P.pmc_launch_shape(e.ctx, P.Request(10, [0], engine=P.PMC_ENGINE_PERSISTENT,
                                                  tally_mode=P.PMC_TALLY_CORE))["core_capacity"]
        entries = np.prod((boxes["hi"] - boxes["lo"]).astype(np.int64), axis=1)
        say("box entries max", int(entries.max()), "capacity", cap)
        if shape == (128, 128, 80):
            assert entries.max() > cap
    finally:
        e.close()


# fields at angles to the grid axes: main axes x, y and z, slopes of both signs
OBLIQUE = ((0.0, -1.0, 0.0), (1.0, 0.0, 0.0), (0.6, -0.8, 0.0), (-0.3, 0.5, 0.81), (0.25, 0.35, -0.9))


@pytest.mark.parametrize("shape", [(64, 64, 40), (128, 128, 80)])
def test_core_mode_oblique_fields(P, shape):
    """Slice cores that follow beams oblique to the grid give tallies
    identical to the plain engine's, for two work-item sizes and over item
    slices."""
    import torch
    ph = W.make_thorax(shape, 0, 10)
    plan = W.plan_thorax(3, n_layers=6, directions=OBLIQUE, n_phases=10)
    plan.spots["phase"] = 0
    wl = W.Workload("thorax_oblique", [ph], plan, 400_000, seed=7)
    e = engine(P, wl)
    try:
        say("core vs plain, oblique fields", shape, len(plan.spots), "spots")
        _, t_plain, _, b_plain = e.dose(wl.n_histories, [0], engine=P.PMC_ENGINE_PLAIN)
        for chunk in (0, 256):
            _, t_c, _, b_c = e.dose(wl.n_histories, [0], engine=P.PMC_ENGINE_PERSISTENT,
                                    tally_mode=P.PMC_TALLY_CORE, chunk=chunk)
            assert np.array_equal(t_c[0], t_plain[0]), chunk
            assert b_c == b_plain
        req = P.Request(wl.n_histories, [0], engine=P.PMC_ENGINE_PERSISTENT, tally_mode=P.PMC_TALLY_CORE,
                        chunk=256)
        n_items = P.pmc_request_items(e.ctx, req)
        tal = torch.zeros(ph.nvox, dtype=torch.int64, device="cuda")
        cnt = torch.zeros(P.PMC_COUNTERS, dtype=torch.int64, device="cuda")
        st = torch.cuda.current_stream()
        cuts = [0, n_items // 3, n_items // 3 + 1, n_items]
        say("oblique core slices", cuts)
        for b, c in zip(cuts, cuts[1:]):
            P.pmc_dose_device(e.ctx, req.slice(b, c), st.cuda_stream, [tal.data_ptr()], cnt.data_ptr())
        torch.cuda.synchronize()
        assert np.array_equal(tal.cpu().numpy(), t_plain[0])
    finally:
        e.close()


def test_core_mode_4d_and_slices(P):
    import torch
    wl = W.workload_thorax4d(n_histories=300_000, shape_xyz=(96, 96, 60))
    e = engine(P, wl)
    phases = list(range(10))
    try:
        say("4D thorax 96x96x60x10 core vs plain")
        _, tp, _, bp = e.dose(wl.n_histories, phases, engine=P.PMC_ENGINE_PLAIN)
        _, tc, _, bc = e.dose(wl.n_histories, phases, engine=P.PMC_ENGINE_PERSISTENT,
                              tally_mode=P.PMC_TALLY_CORE, chunk=500)
        assert bp == bc
        for a, b in zip(tp, tc):
            assert np.array_equal(a, b)
        # three slices of the work items add up to the whole
        req = P.Request(wl.n_histories, phases, engine=P.PMC_ENGINE_PERSISTENT,
                        tally_mode=P.PMC_TALLY_CORE, chunk=500)
        n_items = P.pmc_request_items(e.ctx, req)
        sizes = P.pmc_request_item_histories(e.ctx, req)
        assert len(sizes) == n_items and int(sizes.sum()) == wl.n_histories
        nv = wl.phases[0].nvox
        tal = [torch.zeros(nv, dtype=torch.int64, device="cuda") for _ in phases]
        cnt = torch.zeros(P.PMC_COUNTERS, dtype=torch.int64, device="cuda")
        st = torch.cuda.current_stream()
        cuts = [0, n_items // 3, n_items // 3 + 1, n_items]
        say("core slices", cuts)
        for b, c in zip(cuts, cuts[1:]):
            P.pmc_dose_device(e.ctx, req.slice(b, c), st.cuda_stream, [t.data_ptr() for t in tal],
                              cnt.data_ptr())
        torch.cuda.synchronize()
        for t, ref in zip(tal, tp):
            assert np.array_equal(t.cpu().numpy(), ref)
        # drain signal of the block engine
        flag = torch.zeros(2, dtype=torch.int32, pin_memory=True)
        for t in tal:
            t.zero_()
        P.pmc_dose_device_notify(e.ctx, req, st.cuda_stream, [t.data_ptr() for t in tal], None,
                                 flag.data_ptr() + 4)
        torch.cuda.synchronize()
        assert int(flag[1]) == 1 and int(flag[0]) == 0
        for t, ref in zip(tal, tp):
            assert np.array_equal(t.cpu().numpy(), ref)
    finally:
        e.close()


def test_auto_mode_picks_core_for_large_requests(P):
    """A single-spot request large enough for the block engine: the library
    picks it by itself (the device has LDS for the core) and the tally equals
    the lane engine's."""
    ph = W.make_water(48, 2.5)
    plan = W.plan_single(120.0, 5.0, (0.0, 0.0, 60.0))
    wl = W.Workload("water_single", [ph], plan, 0, seed=11)
    e = engine(P, wl)
    try:
        n = 1024 * 8192 + 5
        req = P.Request(n, [0], engine=P.PMC_ENGINE_PERSISTENT)
        shape = P.pmc_launch_shape(e.ctx, req)
        say("auto shape", shape)
        assert shape["tally_mode"] == P.PMC_TALLY_CORE and shape["core_capacity"] >= 4096
        _, t_auto, _, b_auto = e.dose(n, [0], engine=P.PMC_ENGINE_PERSISTENT)
        _, t_lane, _, b_lane = e.dose(n, [0], engine=P.PMC_ENGINE_PERSISTENT,
                                      tally_mode=P.PMC_TALLY_LANE)
        assert np.array_equal(t_auto[0], t_lane[0]) and b_auto == b_lane
    finally:
        e.close()


def test_core_mode_mixed_calibrations_and_mask(P):
    """Two phases with different HU calibrations in one request (the LUTs stay
    in global memory) and an external mask (vacuum outside the body)."""
    import dataclasses
    base = W.make_thorax((96, 96, 60), 0, 10)
    body = (base.hu > -900).astype(np.uint8)
    ph0 = dataclasses.replace(base, mask=body)
    ph1 = W.scaled_calibration(W.make_thorax((96, 96, 60), 5, 10), 1.035)
    plan = W.plan_thorax(3, n_phases=10)
    plan.spots["phase"] = np.arange(len(plan.spots)) % 2
    wl = W.Workload("mixed", [ph0, ph1], plan, 400_000, seed=9)
    e = engine(P, wl)
    try:
        say("core mode, two calibrations + mask")
        _, tp, _, bp = e.dose(wl.n_histories, [0, 1], engine=P.PMC_ENGINE_PLAIN)
        assert bp["deposited"] + bp["escaped"] + bp["nuclear"] == bp["incident"]
        for mode in (P.PMC_TALLY_LANE, P.PMC_TALLY_CORE):
            _, tc, _, bc = e.dose(wl.n_histories, [0, 1], engine=P.PMC_ENGINE_PERSISTENT,
                                  tally_mode=mode, chunk=300)
            assert bc == bp, mode
            for a, b in zip(tp, tc):
                assert np.array_equal(a, b), mode
        # nothing is deposited outside the mask of phase 0
        assert not tp[0][body.reshape(-1) == 0].any()
    finally:
        e.close()


def test_atomic_log_and_replay(P):
    """The measurement hook of the deposit-address pattern: a logged block-
    engine launch gives the same tallies and counters as the plain one; the
    lanes' logged counts add up to the device-wide atomics the counters
    report; every logged address is an 8-byte slot of one of the request's
    tallies; the replay adds exactly one per replayed entry to the tallies
    (so each replayed atomic hit the logged voxel), with a per-lane cap
    below some lanes' counts."""
    import torch
    wl = W.workload_thorax4d(n_histories=300_000, shape_xyz=(96, 96, 60))
    e = engine(P, wl)
    try:
        phases = [1, 4, 8]
        nv = wl.phases[0].nvox
        st = torch.cuda.current_stream()
        grid = 12
        lanes = grid * 1024
        req = P.Request(wl.n_histories, phases, engine=P.PMC_ENGINE_PERSISTENT, tally_mode=P.PMC_TALLY_CORE,
                        grid_blocks=grid)
        ref = [torch.zeros(nv, dtype=torch.int64, device="cuda") for _ in phases]
        cref = torch.zeros(P.PMC_COUNTERS, dtype=torch.int64, device="cuda")
        P.pmc_dose_device(e.ctx, req, st.cuda_stream, [t.data_ptr() for t in ref], cref.data_ptr())
        tal = [torch.zeros(nv, dtype=torch.int64, device="cuda") for _ in phases]
        cnt = torch.zeros(P.PMC_COUNTERS, dtype=torch.int64, device="cuda")
        cap = 64
        log = torch.zeros(cap * lanes, dtype=torch.int64, device="cuda")
        count = torch.zeros(lanes, dtype=torch.int32, device="cuda")
        say("logged block-engine launch", wl.n_histories, "lanes", lanes)
        P.pmc_atomic_log(e.ctx, req, st.cuda_stream, [t.data_ptr() for t in tal], cnt.data_ptr(),
                         log.data_ptr(), cap, count.data_ptr())
        torch.cuda.synchronize()
        for a, b in zip(tal, ref):
            assert torch.equal(a, b)
        assert torch.equal(cnt, cref)
        c = count.cpu().numpy().astype(np.int64)
        assert c.sum() == int(cnt[12].item()) and c.max() > cap
        n_rep = np.minimum(c, cap)
        lg = log.cpu().numpy().reshape(cap, lanes)
        used = np.arange(cap)[:, None] < n_rep[None, :]
        addr = lg[used].astype(np.uint64)
        base = np.array([t.data_ptr() for t in tal], dtype=np.uint64)
        order = np.argsort(base)
        w = np.searchsorted(base[order], addr, side="right") - 1
        assert np.all(w >= 0)
        which = order[w]
        off = addr - base[which]
        assert np.all(off % 8 == 0) and np.all(off // 8 < nv)
        before = [t.clone() for t in tal]
        say("replay", int(n_rep.sum()), "atomics")
        P.pmc_atomic_replay(e.ctx, st.cuda_stream, log.data_ptr(), cap, count.data_ptr(), lanes)
        torch.cuda.synchronize()
        added = np.zeros(len(phases) * nv, dtype=np.int64)
        np.add.at(added, which.astype(np.int64) * nv + (off // 8).astype(np.int64), 1)
        for i, (a, b) in enumerate(zip(tal, before)):
            assert np.array_equal((a - b).cpu().numpy(), added[i * nv:(i + 1) * nv]), i
        with pytest.raises(P.PmcError):  # the log needs the block engine
            P.pmc_atomic_log(e.ctx, P.Request(1000, [1], engine=P.PMC_ENGINE_PERSISTENT,
                                              tally_mode=P.PMC_TALLY_LANE, grid_blocks=grid),
                             st.cuda_stream, [tal[0].data_ptr()], cnt.data_ptr(), log.data_ptr(), cap,
                             count.data_ptr())
    finally:
        e.close()
