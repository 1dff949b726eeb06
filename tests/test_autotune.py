"""The autotuner's choice on the host (CPU; the transport call is replaced by
a fixed delay per launch shape): the fastest candidate wins, and a preferred
candidate (the library's default shape) is kept when it is within the
tolerance of the fastest, so shapes within timing noise are not picked at
random from run to run."""
import time

from paper_1809_03927_amd import autotune, pmc


def run(monkeypatch, cost, prefer, tolerance):
    def fake(ctx, req, stream, tallies, counters):
        time.sleep(cost[(req.c.block_size, req.c.chunk, req.c.refill_min)])
    monkeypatch.setattr(pmc, "pmc_dose_device", fake)
    cands = [(b, c, r, pmc.PMC_TALLY_CORE) for (b, c, r) in cost]
    return autotune.tune(None, [0], "key", [], 0, 0, lambda: None, 1000, cache_path=None,
                         candidates=cands, repeats=1, prefer=prefer, tolerance=tolerance)


def test_fastest_wins_without_preference(monkeypatch):
    cost = {(1024, 4096, 64): 0.02, (1024, 8192, 64): 0.03, (1024, 16384, 64): 0.05}
    assert run(monkeypatch, cost, None, 0.01)["chunk"] == 4096


def test_preferred_kept_within_tolerance(monkeypatch):
    cost = {(1024, 4096, 64): 0.020, (1024, 8192, 64): 0.0202, (1024, 16384, 64): 0.05}
    best = run(monkeypatch, cost, (1024, 8192, 64, pmc.PMC_TALLY_CORE), 0.25)
    assert best["chunk"] == 8192


def test_preferred_dropped_when_clearly_slower(monkeypatch):
    cost = {(1024, 4096, 64): 0.02, (1024, 8192, 64): 0.021, (1024, 16384, 64): 0.06}
    best = run(monkeypatch, cost, (1024, 16384, 64, pmc.PMC_TALLY_CORE), 0.25)
    assert best["chunk"] in (4096, 8192)
