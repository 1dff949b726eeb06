"""The thorax 4D workload at its full size -- 10 breathing phases of
256x256x160 voxels, 3000 spots, 5e7 histories (the largest count one int64
tally takes) -- in the launch configuration the benchmark times: the
library's default shape for it (block engine, work items of 8192
histories) and its captured graph.

Properties of the whole launch: the energy balance closes exactly; the
integer tallies equal the plain engine's (one launch per phase) and the
graph replay's; a split of the work items adds up to the whole.  Sampled
outputs: the work items of three sampled spots run alone, and their tallies
are compared with the oracle's tallies of exactly those histories (same
keys) -- the history count and incident energy exactly (the FP32 engine's
at the spot energy rounded to FP32), the dose voxel by voxel (voxels above
10 % of the maximum pass if the difference is within 1 % of the maximum or
3 sigma of the difference, sigma = sqrt 2 x the oracle's; same seed, so at
least 99.5 % of them), the total deposited energy within 0.1 %.  The oracle's sigma comes from 50 batches of
the same histories rather than the 10 of the plan-wide check: with 9 degrees
of freedom per voxel a 3-sigma bound alone fails about 1.5 % of the voxels
of two results that agree in distribution (Student's t), with 49 about
0.4 %.  (This test found the FP32 engine depositing 1-6 % too much energy in
air voxels: 98.7 % of one 188 MeV spot's voxels passed, all failures in the
air behind the body.)
"""
import math
import os
import sys

import numpy as np
import pytest

from parity import SAME_SEED_MIN_PASS
from paper_1809_03927_amd import workloads as W

pytestmark = pytest.mark.gpu

CHUNK = 8192


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def full():
    from paper_1809_03927_amd import pmc
    say("thorax4d full size: generating 10 phases of 256x256x160")
    wl = W.workload_thorax4d()
    e = pmc.Engine(device=0, precision=pmc.PMC_FP32, seed=wl.seed)
    e.load_workload(wl)
    yield pmc, wl, e
    e.close()


def total(bal, key):
    return int(bal[key])


def queue_items(per_spot, chunk):
    """(spot, first history, count) of every work item in queue order: the
    first run of every spot with histories (plan order), then every second
    run, and so on."""
    out = []
    r = 0
    while True:
        round_ = [(s, r * chunk, int(min(chunk, per_spot[s] - r * chunk)))
                  for s in range(len(per_spot)) if per_spot[s] > r * chunk]
        if not round_:
            return out
        out += round_
        r += 1


def test_full_size_launch(full):
    import torch
    pmc, wl, e = full
    phases = list(range(10))
    n = wl.n_histories
    req = pmc.Request(n, phases, request_id=wl.request_id, engine=pmc.PMC_ENGINE_PERSISTENT)
    shape = pmc.pmc_launch_shape(e.ctx, req)
    say("default shape", shape)
    assert shape["tally_mode"] == pmc.PMC_TALLY_CORE and shape["chunk"] == CHUNK
    assert shape["block_size"] == 1024
    nv = wl.phases[0].nvox
    say("batched (block engine), 5e7 histories")
    _, t_b, _, b_b = pmc.pmc_dose(e.ctx, req, [nv] * 10, want_dose=False)
    inc = total(b_b, "incident")
    assert total(b_b, "deposited") + total(b_b, "escaped") + total(b_b, "nuclear") == inc
    assert b_b["histories"] == n
    say("plain engine, 10 launches")
    req_p = pmc.Request(n, phases, request_id=wl.request_id, engine=pmc.PMC_ENGINE_PLAIN)
    _, t_p, _, b_p = pmc.pmc_dose(e.ctx, req_p, [nv] * 10, want_dose=False)
    assert b_p == b_b
    for i in phases:
        assert np.array_equal(t_p[i], t_b[i]), i
    del t_p
    # the captured graph the benchmark replays, twice, and a split of the items
    st = torch.cuda.current_stream()
    tal = [torch.zeros(nv, dtype=torch.int64, device="cuda") for _ in phases]
    dose = [torch.zeros(nv, dtype=torch.float64, device="cuda") for _ in phases]
    cnt = torch.zeros(pmc.PMC_COUNTERS, dtype=torch.int64, device="cuda")
    g = pmc.pmc_graph_create(e.ctx, req, [t.data_ptr() for t in tal], cnt.data_ptr(),
                             [d.data_ptr() for d in dose])
    try:
        for replay in range(2):
            say("graph replay", replay)
            pmc.pmc_graph_launch(g, st.cuda_stream, e.ctx)
            torch.cuda.synchronize()
            for i in phases:
                assert np.array_equal(tal[i].cpu().numpy(), t_b[i]), (replay, i)
    finally:
        pmc.pmc_graph_destroy(g)
    n_items = pmc.pmc_request_items(e.ctx, req)
    cut = n_items // 2 + 17
    say("two slices of the work items", n_items, cut)
    for t in tal:
        t.zero_()
    for b, c in ((0, cut), (cut, n_items)):
        pmc.pmc_dose_device(e.ctx, req.slice(b, c), st.cuda_stream, [t.data_ptr() for t in tal],
                            cnt.data_ptr())
    torch.cuda.synchronize()
    for i in phases:
        assert np.array_equal(tal[i].cpu().numpy(), t_b[i]), i


def test_full_size_sampled_spots_against_oracle(full):
    import oracle
    pmc, wl, e = full
    phases = list(range(10))
    n = wl.n_histories
    sp = wl.plan.spots
    req = pmc.Request(n, phases, request_id=wl.request_id, engine=pmc.PMC_ENGINE_PERSISTENT)
    per = pmc.pmc_split_histories(sp, phases, n)
    items = queue_items(per, CHUNK)
    sizes = pmc.pmc_request_item_histories(e.ctx, req)
    assert np.array_equal(sizes, np.array([c for _, _, c in items], dtype=sizes.dtype))
    # three sampled spots: the highest energy of the last phase, the lowest of
    # the first, the median of phase 5
    picks = []
    for ph, how in ((9, np.argmax), (0, np.argmin), (5, None)):
        idx = np.nonzero((sp["phase"] == ph) & (per > 0))[0]
        if how is None:
            order = idx[np.argsort(sp["energy_MeV"][idx], kind="stable")]
            picks.append(int(order[len(order) // 2]))
        else:
            picks.append(int(idx[how(sp["energy_MeV"][idx])]))
    nv = wl.phases[0].nvox
    threads = min(16, os.cpu_count() or 1)
    for s in picks:
        ph = int(sp["phase"][s])
        mine = [k for k, (q, _, _) in enumerate(items) if q == s]
        say(f"spot {s}: phase {ph}, {sp['energy_MeV'][s]:.1f} MeV, {per[s]} histories, items {mine}")
        t_g = np.zeros(nv, dtype=np.int64)
        inc = hist = 0
        for k in mine:
            _, t, _, b = pmc.pmc_dose(e.ctx, req.slice(k, k + 1), [nv] * 10, want_dose=False)
            t_g += t[ph]
            inc += total(b, "incident")
            hist += b["histories"]
            assert sum(int(x.sum()) for i, x in enumerate(t) if i != ph) == 0
        o_t, o_b = oracle.dose_spots(wl.phases, wl.plan, n, wl.seed, s, s + 1, request_id=wl.request_id,
                                     n_threads=threads)
        assert hist == o_b["histories"] == per[s]
        # the FP32 engine starts every proton at the spot energy rounded to
        # FP32 (exactly), the oracle at the FP64 energy
        e_spot = float(sp["energy_MeV"][s])
        e32 = float(np.float32(e_spot))
        assert inc == hist * int(math.ldexp(e32, 32))
        assert total(o_b, "incident") == hist * round(e_spot * 2**32)
        assert abs(inc - total(o_b, "incident")) <= hist * (abs(e32 - e_spot) * 2**32 + 1)
        nb = 50
        s1 = np.zeros(nv)
        s2 = np.zeros(nv)
        for r in range(nb):
            tb, _ = oracle.dose_spots(wl.phases, wl.plan, n, wl.seed, s, s + 1, request_id=wl.request_id,
                                      n_threads=threads, h_mod=nb, h_rem=r)
            x = tb[ph].astype(np.float64)
            s1 += x
            s2 += x * x
        assert np.array_equal(s1.astype(np.int64), o_t[ph])
        _, rho = oracle.convert(wl.phases[ph], np.zeros(nv, dtype=np.int64), 1)
        inv = np.where(rho > 0, 1.0 / np.where(rho > 0, rho, 1.0), 0.0)
        var_b = np.maximum((s2 - s1 * s1 / nb) / (nb - 1), 0.0)
        d_o = s1 * inv
        d_g = t_g.astype(np.float64) * inv
        sig = np.sqrt(2.0 * nb * var_b) * inv
        dmax = d_o.max()
        sel = d_o > 0.1 * dmax
        dd = np.abs(d_g[sel] - d_o[sel])
        frac = float(((dd <= 0.01 * dmax) | (dd <= 3.0 * sig[sel])).mean())
        e_rel = abs(float(t_g.sum()) - float(o_t[ph].sum())) / float(o_t[ph].sum())
        say(f"spot {s}: {int(sel.sum())} voxels above 10 %, pass {frac:.4f}, dE {e_rel:.2e}")
        assert sel.sum() > 100 and frac >= SAME_SEED_MIN_PASS and e_rel <= 1e-3 and math.isfinite(e_rel)


def test_full_size_dim_sampled_voxels(full):
    """Dose interpolation (Eq. (3)) at the benchmark's size and shape: nine
    source phases pulled onto phase 5 through reference-to-source DVFs
    (137 x 97 x 121 points at 2.5 mm), n = 5, by the device entry point.
    Every reference voxel is computed on its own, so the oracle evaluates
    3000 sampled ones (a third of them where the dose is highest) one by one:
    masks identical, doses within 1e-12 relative.  The tallies are seeded
    synthetic ones, so that no input comes from the library."""
    import torch
    import oracle
    import oracle.dim as D
    import oracle.emtm as E
    pmc, wl, e = full
    ref, n = 5, 5
    src = [p for p in range(10) if p != ref]
    tal = [W.random_tally(ph, 100 + i) for i, ph in enumerate(wl.phases)]
    dvfs = {p: W.thorax_dvf(ref, p, n_phases=10) for p in src}
    for p in src:
        pmc.pmc_load_dvf(e.ctx, 300 + p, dvfs[p])
    nv = wl.phases[ref].nvox
    dt = [torch.from_numpy(t).cuda() for t in tal]
    dose = torch.empty(nv, dtype=torch.float64, device="cuda")
    mask = torch.empty(nv, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    say("full-size DIM, 9 sources, n = 5")
    pmc.pmc_accumulate_dim_device(e.ctx, ref, dt[ref].data_ptr(), src, [300 + p for p in src],
                                  [dt[p].data_ptr() for p in src], n, wl.n_histories, 0, dose.data_ptr(),
                                  mask.data_ptr())
    torch.cuda.synchronize()
    got, gmask = dose.cpu().numpy(), mask.cpu().numpy().astype(bool)
    rph = wl.phases[ref]
    want_mask = E.report_mask(rph, [dvfs[p] for p in src])
    assert np.array_equal(gmask, want_mask)
    rho = [oracle.convert(ph, np.zeros(ph.hu.size, dtype=np.int64), 1)[1] for ph in wl.phases]
    doses = [E.phase_dose(t, r, float(np.prod(np.asarray(ph.spacing_mm) * 0.1)), wl.n_histories)
             for ph, t, r in zip(wl.phases, tal, rho)]
    rng = np.random.Generator(np.random.PCG64(17))
    inside = np.nonzero(want_mask)[0]
    top = np.argsort(got)[-1000:]
    pick = np.unique(np.concatenate([rng.choice(inside, 2000, replace=False), top]))
    want = doses[ref][pick].copy()
    for p in src:
        want = want + D.pull(rph, wl.phases[p], doses[p], dvfs[p], n, voxels=pick)
    want = np.where(want_mask[pick], want, 0.0)
    g = got[pick]
    scale = max(float(np.abs(want).max()), 1e-300)
    rel = np.abs(g - want) / np.maximum(np.abs(want), 1e-3 * scale)
    say(f"DIM sampled voxels {len(pick)}: max rel {rel.max():.2e}, identical {np.mean(g == want):.4f}")
    assert rel.max() <= 1e-12
    for p in src:
        pmc.pmc_unload_dvf(e.ctx, 300 + p)


def test_full_size_emtm_separable_and_slab(full):
    """Energy/mass transfer (Eqs. (2), (4)-(6)) at the benchmark's size and
    shape: nine source phases onto phase 5 (source-to-reference DVFs), n = 5,
    device entry point.  Eq. (2) sums independent per-source terms, so the
    nine-source call equals, bit for bit inside its report mask, the
    reference dose plus nine single-source calls added on the host in source
    order; and a 3-slice slab of one source phase (its own phase, zero
    reference tally) against the oracle's push at the full reference size:
    masks identical, doses within 1e-9 relative.  Seeded synthetic tallies."""
    import dataclasses
    import torch
    import oracle
    import oracle.emtm as E
    pmc, wl, e = full
    ref, n = 5, 5
    src = [p for p in range(10) if p != ref]
    tal = [W.random_tally(ph, 200 + i) for i, ph in enumerate(wl.phases)]
    dvfs = {p: W.thorax_dvf(p, ref, n_phases=10) for p in src}
    for p in src:
        pmc.pmc_load_dvf(e.ctx, 100 + p, dvfs[p])
    nv = wl.phases[ref].nvox
    dt = [torch.from_numpy(t).cuda() for t in tal]
    zero = torch.zeros(nv, dtype=torch.int64, device="cuda")
    dose = torch.empty(nv, dtype=torch.float64, device="cuda")
    mask = torch.empty(nv, dtype=torch.uint8, device="cuda")

    def acc(ref_t, sources, tallies):
        pmc.pmc_accumulate_device(e.ctx, ref, ref_t.data_ptr(), sources, [100 + p for p in sources],
                                  [t.data_ptr() for t in tallies], n, wl.n_histories, 0, dose.data_ptr(),
                                  mask.data_ptr())
        torch.cuda.synchronize()
        return dose.cpu().numpy(), mask.cpu().numpy().astype(bool)

    say("full-size EMTM, 9 sources, n = 5")
    full_d, full_m = acc(dt[ref], src, [dt[p] for p in src])
    assert np.array_equal(full_m, E.report_mask(wl.phases[ref], [dvfs[p] for p in src]))
    total, _ = acc(dt[ref], [], [])
    for p in src:
        say("single source", p)
        term, m = acc(zero, [p], [dt[p]])
        assert np.all(m[full_m])
        total = total + term
    assert np.array_equal(full_d[full_m], total[full_m]) and not full_d[~full_m].any()
    # slab of source phase 0 against the oracle
    sp, k = 0, 3
    ph, rph = wl.phases[sp], wl.phases[ref]
    z0 = ph.hu.shape[0] // 2 - 1
    o = (ph.origin_mm[0], ph.origin_mm[1], ph.origin_mm[2] + z0 * ph.spacing_mm[2])
    c = dataclasses.replace(ph, hu=np.ascontiguousarray(ph.hu[z0:z0 + k]), origin_mm=o, mask=None)
    t = np.ascontiguousarray(tal[sp].reshape(ph.hu.shape)[z0:z0 + k]).ravel()
    rho = oracle.convert(c, np.zeros(c.hu.size, dtype=np.int64), 1)[1]
    say("oracle push of a 3-slice slab")
    sums = E.push(c, t, rho, rph, dvfs[sp], n)
    want_mask = E.report_mask(rph, [dvfs[sp]])
    want = np.where(want_mask, E.dose_from_sums(sums, float(np.prod(np.asarray(c.spacing_mm) * 0.1)),
                                                wl.n_histories), 0.0)
    pmc.pmc_load_phase(e.ctx, 200, c)
    try:
        pmc.pmc_load_dvf(e.ctx, 300, dvfs[sp])
        ts = torch.from_numpy(t).cuda()
        pmc.pmc_accumulate_device(e.ctx, ref, zero.data_ptr(), [200], [300], [ts.data_ptr()], n,
                                  wl.n_histories, 0, dose.data_ptr(), mask.data_ptr())
        torch.cuda.synchronize()
        got, gmask = dose.cpu().numpy(), mask.cpu().numpy().astype(bool)
    finally:
        pmc.pmc_unload_phase(e.ctx, 200)
        pmc.pmc_unload_dvf(e.ctx, 300)
    assert np.array_equal(gmask, want_mask)
    sel = want > 0
    rel = np.abs(got[sel] - want[sel]) / want[sel]
    say(f"EMTM slab: {int(sel.sum())} voxels, max rel {rel.max():.2e}, identical {np.mean(got == want):.4f}")
    assert sel.sum() > 1000 and rel.max() <= 1e-9 and not got[~sel].any()
    for p in src:
        pmc.pmc_unload_dvf(e.ctx, 100 + p)


@pytest.mark.parametrize("scenario", ["free", "gated", "repainted"])
def test_full_size_delivery(full, scenario):
    """The delivery simulation (Sec. 2.B, App. A) at the benchmark's size:
    the robust plan's three fields (8000 spots, 600 MU), 25 trials with
    random start phase, breathing period and synchrotron parameters, free,
    gated (phases 3-7) and repainted (0.005 MU per delivery).  Every trial is
    independent, and the oracle replays all 25: MU per spot and phase and
    fill counts identical, end times within 1e-12, except in a timeline with
    a logged near-tie decision (at most one of the 75)."""
    from delivery_check import compare
    from oracle import delivery as OD
    pmc, _, e = full
    plan = W.plan_robust()
    sp = plan.spots.copy()
    sp["weight"] = sp["weight"] / sp["weight"].sum() * 600.0
    kw = {"free": {}, "gated": {"gate_lo": 3, "gate_hi": 7}, "repainted": {"max_mu": 0.005}}[scenario]
    d = W.Delivery(n_trials=25, period_sd_s=0.4, period_min_s=3, period_max_s=7, seed=17, **kw)
    say("full-size delivery", scenario)
    got = pmc.pmc_delivery_simulate(e.ctx, d, sp, len(plan.fields))
    want = OD.simulate(sp, len(plan.fields), d)
    flips = compare(got, want, sp, len(plan.fields), max_flips=1)
    say(f"full-size delivery {scenario}: {flips} timelines with a flipped near-tie decision")
    # MU conserved per spot and trial
    assert np.allclose(got["mu"].sum(axis=2), sp["weight"][None, :], rtol=1e-12, atol=0)


@pytest.mark.parametrize("name", ["liver", "esophagus"])
def test_case_phantom_full_size_equals_plain(name):
    """A patient-shaped case at the benchmark's size (5e7 histories over ten
    phases, fields oblique to the grid: the block engine's slice cores):
    batched tallies and balance equal the plain engine's."""
    from paper_1809_03927_amd import pmc
    say(f"case {name}: generating")
    wl = W.workload_case(name)
    e = pmc.Engine(device=0, precision=pmc.PMC_FP32, seed=wl.seed)
    try:
        e.load_workload(wl)
        phases = list(range(len(wl.phases)))
        req = pmc.Request(wl.n_histories, phases, request_id=wl.request_id, engine=pmc.PMC_ENGINE_PERSISTENT)
        shape = pmc.pmc_launch_shape(e.ctx, req)
        assert shape["tally_mode"] == pmc.PMC_TALLY_CORE
        nv = [ph.nvox for ph in wl.phases]
        say(f"case {name}: batched")
        _, t_b, _, b_b = pmc.pmc_dose(e.ctx, req, nv, want_dose=False)
        assert b_b["deposited"] + b_b["escaped"] + b_b["nuclear"] == b_b["incident"]
        say(f"case {name}: plain")
        req_p = pmc.Request(wl.n_histories, phases, request_id=wl.request_id, engine=pmc.PMC_ENGINE_PLAIN)
        _, t_p, _, b_p = pmc.pmc_dose(e.ctx, req_p, nv, want_dose=False)
        assert b_p == b_b
        for i in phases:
            assert np.array_equal(t_p[i], t_b[i]), i
    finally:
        e.close()
