"""Pin of the history split (histories per spot proportional to weight, largest
remainder, ties to the lower spot index) against exact rational arithmetic."""
from fractions import Fraction

import numpy as np
import pytest

from paper_1809_03927_amd import workloads as W


def hamilton_exact(weights, n):
    W_ = sum(Fraction(w) for w in weights)
    q = [Fraction(w) * n / W_ for w in weights]
    fl = [int(x) for x in q]  # floor: all non-negative
    rem = sorted(range(len(q)), key=lambda i: (-(q[i] - fl[i]), i))
    left = n - sum(fl)
    for i in rem[:left]:
        fl[i] += 1
    return fl


def spots_with(weights, phases=None):
    s = np.zeros(len(weights), dtype=W.SPOT_DTYPE)
    s["weight"] = weights
    s["energy_MeV"] = 100.0
    s["phase"] = 0 if phases is None else phases
    return s


@pytest.mark.parametrize("seed", range(6))
def test_split_matches_exact_hamilton(orc, seed):
    rng = np.random.default_rng(seed)
    m = int(rng.integers(1, 60))
    # dyadic weights: exact in binary floating point, so the two agree exactly
    w = rng.integers(1, 1 << 12, size=m).astype(float) / 64.0
    n = int(rng.integers(1, 10_000))
    got = orc.split_histories(spots_with(w), [0], n)
    assert got.sum() == n
    assert list(got) == hamilton_exact(list(w), n)


def test_split_lognormal_properties(orc):
    plan = W.plan_slabs(2)
    n = 10_000_000
    got = orc.split_histories(plan.spots, [0], n)
    q = n * plan.spots["weight"] / plan.spots["weight"].sum()
    assert got.sum() == n and np.all(np.abs(got - q) < 1.0)


def test_split_only_listed_phases_and_ties(orc):
    s = spots_with([1.0, 1.0, 1.0, 5.0], phases=[0, 1, 0, 2])
    got = orc.split_histories(s, [0, 1], 4)
    # three equal spots share 4: the extra one goes to the lowest index
    assert list(got) == [2, 1, 1, 0]
    assert list(orc.split_histories(s, [2], 3)) == [0, 0, 0, 3]


def test_spot_selection_and_batches_partition_the_histories(orc):
    """The per-spot selection takes exactly the spots' histories of the whole
    request's split, and its h % h_mod batches partition them."""
    wl = W.workload_slabs()
    n = 20_000
    whole, b_all = orc.dose(wl.phases, wl.plan, n, wl.seed)[0::2]
    per = orc.split_histories(wl.plan.spots, [0], n)
    parts = [orc.dose_spots(wl.phases, wl.plan, n, wl.seed, a, b) for a, b in ((0, 7), (7, 300), (300, 500))]
    assert sum(p[1]["histories"] for p in parts) == n
    assert np.array_equal(sum(p[0][0] for p in parts), whole[0])
    t, b = orc.dose_spots(wl.phases, wl.plan, n, wl.seed, 3, 5)
    assert b["histories"] == int(per[3] + per[4])
    batches = [orc.dose_spots(wl.phases, wl.plan, n, wl.seed, 3, 5, h_mod=3, h_rem=r) for r in range(3)]
    assert np.array_equal(sum(x[0][0] for x in batches), t[0])
    assert sum(x[1]["incident"] for x in batches) == b["incident"]
