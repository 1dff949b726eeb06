"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, validates arguments before any device work (using a
validation-only context, device = -1) and computes the history split exactly
as the oracle does."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1809_03927_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def P():
    from paper_1809_03927_amd import pmc
    if not os.path.exists(pmc.LIB_PATH):
        from paper_1809_03927_amd import build
        build.build()
    return pmc


def header_functions():
    txt = open(os.path.join(ROOT, "include", "pmc.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(pmc_[a-z_]+)\s*\(", txt, re.M)))


def test_library_exports_every_header_symbol(P):
    names = header_functions()
    assert len(names) >= 19
    lib = P.lib()  # loads the HIP runtime the way the binding does
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(P.EXPORTS) == names


def test_struct_layouts_match_header(P):
    assert C.sizeof(P.pmc_config) == 24
    assert C.sizeof(P.pmc_request) == 72
    assert C.sizeof(P.pmc_shape) == 32
    assert C.sizeof(P.pmc_balance) == 8 * 16
    assert W.SPOT_DTYPE.itemsize == 48 and W.FIELD_DTYPE.itemsize == 72
    assert P.TRACE_DTYPE.itemsize == 120


@pytest.fixture()
def vctx(P):
    ctx = P.pmc_create(device=-1)
    yield ctx
    P.pmc_destroy(ctx)


def test_create_rejects_bad_config(P):
    with pytest.raises(P.PmcError) as e:
        P.pmc_create(device=-1, precision=7)
    assert e.value.code == P.PMC_E_INVAL
    assert "precision" in P.pmc_last_error(None)
    P.pmc_destroy(None)  # NULL-safe


def test_load_phase_validation(P, vctx):
    ph = W.make_water(8, 2.0)
    P.pmc_load_phase(vctx, 0, ph)  # valid
    bad = W.make_water(8, 2.0)
    bad.calib_hu = np.array([0.0, 0.0])
    bad.calib_rho = np.array([1.0, 1.0])
    bad.calib_rsp = np.array([1.0, 1.0])
    with pytest.raises(P.PmcError) as e:
        P.pmc_load_phase(vctx, 1, bad)
    assert e.value.code == P.PMC_E_INVAL and "increasing" in str(e.value)
    bad = W.make_water(8, 2.0)
    bad.spacing_mm = (2.0, 0.0, 2.0)
    with pytest.raises(P.PmcError):
        P.pmc_load_phase(vctx, 1, bad)
    bad = W.make_water(8, 2.0)
    bad.calib_rho = bad.calib_rho.copy()
    bad.calib_rho[0] = np.nan
    with pytest.raises(P.PmcError):
        P.pmc_load_phase(vctx, 1, bad)
    with pytest.raises(P.PmcError):
        P.pmc_load_phase(vctx, 5000, ph)


def test_load_spots_validation(P, vctx):
    plan = W.plan_single(150.0, 5.0)
    P.pmc_load_spots(vctx, plan.fields, plan.spots)
    for field, val in [("energy_MeV", 0.5), ("energy_MeV", 301.0), ("weight", 0.0),
                       ("sigma_mm", -1.0), ("field", 3), ("energy_MeV", np.nan)]:
        s = plan.spots.copy()
        s[field] = val
        with pytest.raises(P.PmcError) as e:
            P.pmc_load_spots(vctx, plan.fields, s)
        assert e.value.code == P.PMC_E_INVAL
    f = plan.fields.copy()
    f["bev_u"] = (0.0, 0.0, 1.0)  # parallel to the beam
    with pytest.raises(P.PmcError):
        P.pmc_load_spots(vctx, f, plan.spots)


def test_dose_validation_order(P, vctx):
    req = P.Request(1000, [0])
    with pytest.raises(P.PmcError) as e:
        P.pmc_dose(vctx, req, [8 ** 3])
    assert e.value.code == P.PMC_E_STATE  # no plan yet
    plan = W.plan_single(150.0, 5.0)
    P.pmc_load_spots(vctx, plan.fields, plan.spots)
    with pytest.raises(P.PmcError) as e:
        P.pmc_dose(vctx, req, [8 ** 3])
    assert e.value.code == P.PMC_E_NOPHASE
    P.pmc_load_phase(vctx, 0, W.make_water(8, 2.0))
    with pytest.raises(P.PmcError) as e:
        P.pmc_dose(vctx, P.Request(P.PMC_MAX_HISTORIES + 1, [0]), [8 ** 3])
    assert e.value.code == P.PMC_E_RANGE
    with pytest.raises(P.PmcError) as e:
        P.pmc_dose(vctx, P.Request(0, [0]), [8 ** 3])
    assert e.value.code == P.PMC_E_INVAL
    with pytest.raises(P.PmcError) as e:
        P.pmc_dose(vctx, P.Request(10, [0, 0]), [8 ** 3, 8 ** 3])
    assert e.value.code == P.PMC_E_INVAL
    with pytest.raises(P.PmcError) as e:
        P.pmc_dose(vctx, P.Request(10, [0], block_size=100), [8 ** 3])
    assert e.value.code == P.PMC_E_INVAL
    # all arguments valid: the validation-only context reports the missing device
    with pytest.raises(P.PmcError) as e:
        P.pmc_dose(vctx, req, [8 ** 3])
    assert e.value.code == P.PMC_E_DEVICE
    P.pmc_unload_phase(vctx, 0)
    with pytest.raises(P.PmcError) as e:
        P.pmc_unload_phase(vctx, 0)
    assert e.value.code == P.PMC_E_NOPHASE


def test_launch_shape_defaults(P):
    """Lane mode: work items shrink for small requests so that every resident
    wave (16 per compute unit, 256 units assumed without a device) gets about
    four of them.  Core mode once the work items (a spot's partial last item
    counted with its full ones) average at least one history per lane of a
    1024-thread block; its items hold 8192 histories, halved down to 1024
    while the request has fewer than that per compute unit.  Explicit values
    pass through."""
    ctx = P.pmc_create(device=-1)
    pers, lane, core = P.PMC_ENGINE_PERSISTENT, P.PMC_TALLY_LANE, P.PMC_TALLY_CORE
    try:
        plan = W.plan_single(150.0, 5.0)
        P.pmc_load_spots(ctx, plan.fields, plan.spots)
        P.pmc_load_phase(ctx, 0, W.make_water(8, 2.0))
        waves = 16 * 256
        for n, chunk in [(1, 64), (4 * waves * 128 - 1, 64), (4 * waves * 128, 128),
                         (4 * waves * 256 - 1, 128), (4 * waves * 256, 256)]:
            got = P.pmc_launch_shape(ctx, P.Request(n, [0], engine=pers, tally_mode=lane))
            assert got == {"block_size": 1024, "chunk": chunk, "refill_min": 64, "tally_mode": lane,
                           "core_capacity": 0}, n
        # one spot: core mode from 1024 histories on, items of 1024 up to 8192
        # per compute unit, then of 8192
        for n, chunk in [(1024, 1024), (100_000, 1024), (2048 * 256 - 1, 1024), (2048 * 256, 2048),
                         (8192 * 256 - 1, 4096), (8192 * 256, 8192), (P.PMC_MAX_HISTORIES, 8192)]:
            got = P.pmc_launch_shape(ctx, P.Request(n, [0], engine=pers))
            assert got["tally_mode"] == core and got["chunk"] == chunk and got["block_size"] == 1024, (n, got)
            assert got["core_capacity"] > 4096
        assert P.pmc_launch_shape(ctx, P.Request(1023, [0], engine=pers))["tally_mode"] == lane
        # forced modes, explicit shapes
        assert P.pmc_launch_shape(ctx, P.Request(10, [0], engine=pers, tally_mode=core))["chunk"] == 1024
        assert P.pmc_launch_shape(ctx, P.Request(10**7, [0], engine=pers, tally_mode=core))["chunk"] == 8192
        assert P.pmc_launch_shape(ctx, P.Request(P.PMC_MAX_HISTORIES, [0], engine=pers,
                                                 tally_mode=lane))["tally_mode"] == lane
        assert P.pmc_launch_shape(ctx, P.Request(P.PMC_MAX_HISTORIES, [0], engine=pers,
                                                 block_size=512))["tally_mode"] == lane
        got = P.pmc_launch_shape(ctx, P.Request(10, [0], engine=pers, block_size=512, chunk=7,
                                                refill_min=3))
        assert (got["block_size"], got["chunk"], got["refill_min"]) == (512, 7, 3)
        assert P.pmc_launch_shape(ctx, P.Request(10, [0])) == {
            "block_size": 256, "chunk": 0, "refill_min": 0, "tally_mode": 0, "core_capacity": 0}
        for bad in (dict(block_size=100), dict(engine=pers, tally_mode=3),
                    dict(engine=pers, tally_mode=core, block_size=512), dict(tally_mode=core)):
            with pytest.raises(P.PmcError) as e:
                P.pmc_launch_shape(ctx, P.Request(10, [0], **bad))
            assert e.value.code == P.PMC_E_INVAL, bad
        # many spots: items are whole spots here, core mode once they average 1024 histories
        plan = W.plan_thorax(3, n_layers=4, grid=(15, 10), n_phases=1)
        assert len(plan.spots) == 600
        P.pmc_load_spots(ctx, plan.fields, plan.spots)
        assert P.pmc_launch_shape(ctx, P.Request(600 * 1024 - 1, [0], engine=pers))["tally_mode"] == lane
        assert P.pmc_launch_shape(ctx, P.Request(600 * 1024, [0], engine=pers))["tally_mode"] == core
    finally:
        P.pmc_destroy(ctx)
    ctx = P.pmc_create(device=-1, precision=P.PMC_FP64)
    try:
        plan = W.plan_single(150.0, 5.0)
        P.pmc_load_spots(ctx, plan.fields, plan.spots)
        P.pmc_load_phase(ctx, 0, W.make_water(8, 2.0))
        assert P.pmc_launch_shape(ctx, P.Request(P.PMC_MAX_HISTORIES, [0], engine=pers)) == {
            "block_size": 256, "chunk": 256, "refill_min": 64, "tally_mode": lane, "core_capacity": 0}
        for bad in (dict(block_size=512), dict(engine=pers, tally_mode=core)):
            with pytest.raises(P.PmcError) as e:
                P.pmc_launch_shape(ctx, P.Request(10, [0], **bad))
            assert e.value.code == P.PMC_E_INVAL
    finally:
        P.pmc_destroy(ctx)


@pytest.mark.parametrize("wl_name", ["slabs", "thorax"])
def test_split_matches_oracle(P, orc, wl_name):
    plan = W.plan_slabs(2) if wl_name == "slabs" else W.plan_thorax(3)
    phases = sorted(set(plan.spots["phase"].tolist()))
    for n in (1, 7, 12345, 10_000_000, 50_000_000):
        a = P.pmc_split_histories(plan.spots, phases, n)
        b = orc.split_histories(plan.spots, phases, n)
        assert np.array_equal(a, b) and a.sum() == n
    sub = phases[:3]
    assert np.array_equal(P.pmc_split_histories(plan.spots, sub, 99_999),
                          orc.split_histories(plan.spots, sub, 99_999))


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_1809_03927_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".hpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "pmc_oracle" not in txt and "liboracle" not in txt, f


def test_one_hip_runtime_in_the_process(P):
    """libpmc and PyTorch share one HIP runtime (two copies in one process
    leave the second without a device)."""
    P.lib()
    import torch  # noqa: F401
    paths = set()
    with open("/proc/self/maps") as f:
        for line in f:
            if "libamdhip64" in line:
                paths.add(line.split()[-1])
    assert len(paths) == 1, paths


def test_balance_from_words_matches_library(P):
    """The binding's decoding of a counter block read back earlier equals the
    library's pmc_balance_from_counters."""
    ctx = P.pmc_create(device=-1)
    try:
        plan = W.plan_single(150.0, 5.0)
        P.pmc_load_spots(ctx, plan.fields, plan.spots)
        P.pmc_load_phase(ctx, 0, W.make_water(8, 2.0))
        req = P.Request(12345, [0], engine=P.PMC_ENGINE_PERSISTENT)
        rng = np.random.default_rng(3)
        c = rng.integers(0, 2**63, size=P.PMC_COUNTERS, dtype=np.uint64)
        c[[1, 3, 5]] = [0, 7, 1]
        dep = (5 << 64) + 99
        ref = P.pmc_balance_from_counters(ctx, req, c, dep)
        inc = P.pmc_balance_from_counters(ctx, req, np.zeros(P.PMC_COUNTERS), 0)["incident"]
        assert P.balance_from_words(c, dep, inc) == ref
    finally:
        P.pmc_destroy(ctx)


def test_slice_incident_energy_is_the_slices(P):
    """The incident energy of a slice of a persistent-engine request counts
    only its work items: the slices of a partition add up to the whole, and a
    slice of one spot's items is that spot's share.  Host-only (a
    validation-only context)."""
    ctx = P.pmc_create(device=-1)
    try:
        wl = W.workload_slabs()
        P.pmc_load_spots(ctx, wl.plan.fields, wl.plan.spots)
        P.pmc_load_phase(ctx, 0, wl.phases[0])
        n = 1_000_003
        req = P.Request(n, [0], engine=P.PMC_ENGINE_PERSISTENT, chunk=700)
        zero = np.zeros(P.PMC_COUNTERS)
        whole = P.pmc_balance_from_counters(ctx, req, zero, 0)["incident"]
        sizes = P.pmc_request_item_histories(ctx, req)
        m = len(sizes)
        cuts = [0, 1, 37, m // 2, m - 1, m]
        parts = [P.pmc_balance_from_counters(ctx, req.slice(a, b), zero, 0)["incident"]
                 for a, b in zip(cuts, cuts[1:])]
        assert all(x > 0 for x in parts) and sum(parts) == whole
        # open-ended slice [k, end) and the whole request as (0, 0)
        tail = P.pmc_balance_from_counters(ctx, req.slice(m // 2, 0), zero, 0)["incident"]
        assert tail == sum(parts[3:])
        # one item: its histories times the spot's incident energy per history
        per = P.pmc_split_histories(wl.plan.spots, [0], n)
        first = P.pmc_balance_from_counters(ctx, req.slice(0, 1), zero, 0)["incident"]
        s0 = int(np.nonzero(per)[0][0])
        assert first % int(sizes[0]) == 0 and first // int(sizes[0]) > 0
        assert int(sizes[0]) == min(700, int(per[s0]))
    finally:
        P.pmc_destroy(ctx)


def test_dvf_and_accumulation_validation(P):
    ctx = P.pmc_create(device=-1)
    try:
        ph = W.make_water(8, 2.0)
        P.pmc_load_phase(ctx, 0, ph)
        P.pmc_load_phase(ctx, 1, ph)
        n = (3, 3, 3)
        good = W.Dvf(n, (0.0, 0.0, 0.0), (4.0, 4.0, 4.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0),
                     np.zeros((3, 3, 3, 3)))
        for bad in (W.Dvf((1, 3, 3), good.start_mm, good.spacing_mm, good.row, good.col, np.zeros((3, 3, 1, 3))),
                    W.Dvf(n, good.start_mm, (4.0, 0.0, 4.0), good.row, good.col, good.delta_mm),
                    W.Dvf(n, good.start_mm, good.spacing_mm, good.row, (1.0, 0.0, 0.0), good.delta_mm),
                    W.Dvf(n, good.start_mm, good.spacing_mm, good.row, good.col,
                          np.full((3, 3, 3, 3), np.nan))):
            with pytest.raises(P.PmcError) as e:
                P.pmc_load_dvf(ctx, 0, bad)
            assert e.value.code == P.PMC_E_INVAL
        P.pmc_load_dvf(ctx, 4, good)
        t = np.zeros(8 ** 3, dtype=np.int64)
        with pytest.raises(P.PmcError) as e:
            P.pmc_accumulate(ctx, 0, t, [1], [5], [t], 2, 10, 8 ** 3)
        assert e.value.code == P.PMC_E_STATE  # dvf 5 not loaded
        with pytest.raises(P.PmcError) as e:
            P.pmc_accumulate(ctx, 0, t, [2], [4], [t], 2, 10, 8 ** 3)
        assert e.value.code == P.PMC_E_NOPHASE
        for kw in (dict(n_sub=0), dict(n_sub=17), dict(n_histories=0)):
            args = dict(n_sub=2, n_histories=10)
            args.update(kw)
            with pytest.raises(P.PmcError) as e:
                P.pmc_accumulate(ctx, 0, t, [1], [4], [t], args["n_sub"], args["n_histories"], 8 ** 3)
            assert e.value.code == P.PMC_E_INVAL, kw
        with pytest.raises(P.PmcError) as e:
            P.pmc_accumulate(ctx, 0, t, [1], [4], [t], 2, 10, 8 ** 3)
        assert e.value.code == P.PMC_E_DEVICE  # all arguments valid
        # the same checks for dose interpolation
        with pytest.raises(P.PmcError) as e:
            P.pmc_accumulate_dim(ctx, 0, t, [1], [5], [t], 2, 10, 8 ** 3)
        assert e.value.code == P.PMC_E_STATE
        with pytest.raises(P.PmcError) as e:
            P.pmc_accumulate_dim(ctx, 0, t, [1], [4], [t], 17, 10, 8 ** 3)
        assert e.value.code == P.PMC_E_INVAL
        with pytest.raises(P.PmcError) as e:
            P.pmc_accumulate_dim(ctx, 0, t, [1], [4], [t], 3, 10, 8 ** 3)
        assert e.value.code == P.PMC_E_DEVICE
        with pytest.raises(P.PmcError) as e:
            P.pmc_dvf_points(ctx, 4, n)
        assert e.value.code == P.PMC_E_DEVICE
        with pytest.raises(P.PmcError) as e:
            P.pmc_dvf_points(ctx, 9, n)
        assert e.value.code == P.PMC_E_STATE
        # rigid matrices of Eq. (7): accepted when rigid, rejected otherwise
        rot = np.eye(4)
        rot[:2, :2] = [[0.6, -0.8], [0.8, 0.6]]
        rot[:3, 3] = [1.0, -2.0, 3.0]
        P.pmc_load_dvf(ctx, 6, W.Dvf(n, good.start_mm, good.spacing_mm, good.row, good.col, good.delta_mm,
                                     pre=rot, post=np.linalg.inv(rot)))
        stretched = np.eye(4)
        stretched[0, 0] = 1.1
        for m in (stretched, np.diag([1.0, 1.0, 1.0, 2.0]), np.full((4, 4), np.nan)):
            with pytest.raises(P.PmcError) as e:
                P.pmc_load_dvf(ctx, 7, W.Dvf(n, good.start_mm, good.spacing_mm, good.row, good.col,
                                             good.delta_mm, post=m))
            assert e.value.code == P.PMC_E_INVAL
        P.pmc_unload_dvf(ctx, 4)
        with pytest.raises(P.PmcError):
            P.pmc_unload_dvf(ctx, 4)
    finally:
        P.pmc_destroy(ctx)


def test_delivery_validation(P):
    """Invalid delivery options or spots are rejected before any device work;
    valid ones reach the device check of a validation-only context."""
    ctx = P.pmc_create(device=-1)
    try:
        plan = W.plan_thorax(3, n_phases=10)
        sp = plan.spots.copy()
        sp["weight"] = sp["weight"] / sp["weight"].sum() * 300.0
        with pytest.raises(P.PmcError) as e:
            P.pmc_delivery_simulate(ctx, W.Delivery(n_trials=2), sp, len(plan.fields))
        assert e.value.code == P.PMC_E_DEVICE
        for bad in (dict(n_phases=0), dict(n_phases=65), dict(start_phase=10), dict(gate_lo=3, gate_hi=2),
                    dict(gate_lo=0, gate_hi=10), dict(max_mu=-1.0), dict(n_trials=0), dict(period_s=0.0),
                    dict(period_sd_s=-1.0), dict(period_min_s=-1)):
            with pytest.raises(P.PmcError) as e:
                P.pmc_delivery_simulate(ctx, W.Delivery(**bad), sp, 1)
            assert e.value.code == P.PMC_E_INVAL, bad
        # a spill rate that a draw within 6 sigma could make non-positive
        sync = dict(W.SYNC_DEFAULT)
        sync["spill_rate_mu_s"] = (1.0, 0.5)
        with pytest.raises(P.PmcError) as e:
            P.pmc_delivery_simulate(ctx, W.Delivery(sync=sync), sp, 1)
        assert e.value.code == P.PMC_E_INVAL
        bad_sp = sp.copy()
        bad_sp["field"][5] = 3
        with pytest.raises(P.PmcError) as e:
            P.pmc_delivery_simulate(ctx, W.Delivery(), bad_sp, 1)
        assert e.value.code == P.PMC_E_INVAL
        bad_sp = sp.copy()
        bad_sp["weight"][0] = 0.0
        with pytest.raises(P.PmcError) as e:
            P.pmc_delivery_simulate(ctx, W.Delivery(), bad_sp, 1)
        assert e.value.code == P.PMC_E_INVAL
    finally:
        P.pmc_destroy(ctx)
