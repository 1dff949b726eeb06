"""Captured graphs and the autotuner, through the C ABI on device buffers.

A graph replay must equal an eager run bit for bit, on every replay, with
unrelated eager work and synchronisations between replays; the autotuner
must return one of its candidates, and every candidate gives the same tally.
"""
import sys

import numpy as np
import pytest

from paper_1809_03927_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def setup():
    import torch
    from paper_1809_03927_amd import pmc
    wl = W.workload_thorax4d(n_histories=400_000, shape_xyz=(96, 96, 60))
    e = pmc.Engine(device=0, seed=wl.seed)
    e.load_workload(wl)
    yield torch, pmc, wl, e
    e.close()


def buffers(torch, wl):
    nv = wl.phases[0].nvox
    t = [torch.zeros(nv, dtype=torch.int64, device="cuda") for _ in wl.phases]
    d = [torch.zeros(nv, dtype=torch.float64, device="cuda") for _ in wl.phases]
    c = torch.zeros(16, dtype=torch.int64, device="cuda")
    return t, d, c


def test_graph_replays_equal_eager(setup):
    torch, pmc, wl, e = setup
    phases = list(range(10))
    st = torch.cuda.current_stream()
    req = pmc.Request(wl.n_histories, phases, engine=pmc.PMC_ENGINE_PERSISTENT)
    # eager reference
    t_ref, d_ref, c_ref = buffers(torch, wl)
    pmc.pmc_dose_device(e.ctx, req, st.cuda_stream, [t.data_ptr() for t in t_ref], c_ref.data_ptr())
    for i, p in enumerate(phases):
        pmc.pmc_convert_device(e.ctx, p, t_ref[i].data_ptr(), wl.n_histories, st.cuda_stream,
                               d_ref[i].data_ptr(), None)
    torch.cuda.synchronize()
    t_g, d_g, c_g = buffers(torch, wl)
    for t in t_g:  # garbage that the graph must clear
        t.fill_(12345)
    c_g.fill_(7)
    g = pmc.pmc_graph_create(e.ctx, req, [t.data_ptr() for t in t_g], c_g.data_ptr(),
                             [d.data_ptr() for d in d_g])
    t_x, _, c_x = buffers(torch, wl)
    other = pmc.Request(50_000, [3], engine=pmc.PMC_ENGINE_PLAIN, request_id=9)
    for replay in range(4):
        say("graph replay", replay)
        pmc.pmc_graph_launch(g, st.cuda_stream, e.ctx)
        torch.cuda.synchronize()
        for a, b in zip(t_g, t_ref):
            assert torch.equal(a, b), replay
        for a, b in zip(d_g, d_ref):
            assert torch.equal(a, b), replay
        assert torch.equal(c_g[:13], c_ref[:13])
        # unrelated eager work on the same context between replays
        for t in t_x:
            t.zero_()
        pmc.pmc_dose_device(e.ctx, other, st.cuda_stream, [t_x[3].data_ptr()], c_x.data_ptr())
        torch.cuda.synchronize()
    pmc.pmc_graph_destroy(g)


def test_graph_refuses_a_replaced_phase(setup):
    """A graph reads its phases' device grids by address: after one of them
    is replaced (pmc_load_phase on its id) or unloaded, the replay is
    refused with PMC_E_STATE and nothing runs (the tallies keep the marker
    the replay would have cleared); a graph captured afterwards runs."""
    torch, pmc, wl, e = setup
    st = torch.cuda.current_stream()
    req = pmc.Request(50_000, [2, 3], engine=pmc.PMC_ENGINE_PERSISTENT)
    t_g, d_g, c_g = buffers(torch, wl)
    g = pmc.pmc_graph_create(e.ctx, req, [t_g[0].data_ptr(), t_g[1].data_ptr()], c_g.data_ptr(), None)
    try:
        pmc.pmc_graph_launch(g, st.cuda_stream, e.ctx)
        torch.cuda.synchronize()
        first = t_g[1].clone()
        say("graph after a phase reload")
        pmc.pmc_load_phase(e.ctx, 3, wl.phases[3])  # same content, new device memory
        t_g[0].fill_(777)
        t_g[1].fill_(777)
        with pytest.raises(pmc.PmcError) as ex:
            pmc.pmc_graph_launch(g, st.cuda_stream, e.ctx)
        assert ex.value.code == pmc.PMC_E_STATE
        torch.cuda.synchronize()
        assert bool((t_g[0] == 777).all()) and bool((t_g[1] == 777).all())
    finally:
        pmc.pmc_graph_destroy(g)
    g = pmc.pmc_graph_create(e.ctx, req, [t_g[0].data_ptr(), t_g[1].data_ptr()], c_g.data_ptr(), None)
    try:
        pmc.pmc_graph_launch(g, st.cuda_stream, e.ctx)
        torch.cuda.synchronize()
        assert torch.equal(t_g[1], first)
        say("graph after unloading a phase")
        pmc.pmc_unload_phase(e.ctx, 2)
        with pytest.raises(pmc.PmcError) as ex:
            pmc.pmc_graph_launch(g, st.cuda_stream, e.ctx)
        assert ex.value.code == pmc.PMC_E_STATE
    finally:
        pmc.pmc_graph_destroy(g)
        pmc.pmc_load_phase(e.ctx, 2, wl.phases[2])


def test_autotune_candidates_identical(setup, tmp_path):
    torch, pmc, wl, e = setup
    from paper_1809_03927_amd import autotune
    phases = list(range(10))
    st = torch.cuda.current_stream()
    t, _, c = buffers(torch, wl)
    cands = [(256, 64, 64), (512, 256, 32), (1024, 1024, 48)]
    best = autotune.tune(e.ctx, phases, "test-key", [x.data_ptr() for x in t], c.data_ptr(),
                         st.cuda_stream, torch.cuda.synchronize, 100_000,
                         cache_path=str(tmp_path / "tune.json"), candidates=cands, repeats=1)
    assert (best["block_size"], best["chunk"], best["refill_min"]) in cands
    again = autotune.tune(e.ctx, phases, "test-key", [x.data_ptr() for x in t], c.data_ptr(),
                          st.cuda_stream, torch.cuda.synchronize, 100_000,
                          cache_path=str(tmp_path / "tune.json"), candidates=[(64, 1, 1)])
    assert again == best  # served from the cache
    ref = None
    for blk, ch, rf in cands:
        for x in t:
            x.zero_()
        req = pmc.Request(200_000, phases, engine=pmc.PMC_ENGINE_PERSISTENT, block_size=blk,
                          chunk=ch, refill_min=rf)
        pmc.pmc_dose_device(e.ctx, req, st.cuda_stream, [x.data_ptr() for x in t], c.data_ptr())
        torch.cuda.synchronize()
        cur = [x.cpu().numpy() for x in t]
        if ref is None:
            ref = cur
        else:
            assert all(np.array_equal(a, b) for a, b in zip(ref, cur)), (blk, ch, rf)
