"""The FP32 dose criterion against the FP64 oracle and its pass-fraction bars.

Criterion (per voxel, on tallies of equal history counts; dose is a
per-voxel scaling of the tally): a voxel whose oracle value is above 10 % of
the maximum passes if |dD| <= 1 % of the maximum or |dD| <= 3 sigma_diff,
sigma_diff = sqrt(2) x the oracle's per-voxel standard deviation from
history batches (history index mod n_batches).

"Within 3 sigma in every voxel" cannot hold literally for a statistical
estimate over thousands of voxels: even two runs of the oracle itself with
independent seeds fail a fraction of them.  So the bar is a pass fraction:

* independent seeds (a purely statistical comparison): at least the
  fraction two oracle runs reach at the same history and batch counts,
  minus 3 standard errors (tests/golden/pass_fractions.json, written by
  tests/golden/make_pass_fractions.py from oracle runs only);
* the oracle's own seed (FP32 and FP64 share their random numbers, so a
  history follows the same path until a decision differs): at least
  SAME_SEED_MIN_PASS.
"""
import json
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SAME_SEED_MIN_PASS = 0.995


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def oracle_with_sigma(orc, wl, n, n_batches=100, seed=None):
    """Oracle tally (first phase), its per-voxel standard deviation and the
    standard deviation of its total, from history batches (history index mod
    n_batches), accumulated one batch at a time."""
    seed = wl.seed if seed is None else seed
    tot = sq = None
    totals = []
    for b in range(n_batches):
        t, _ = orc.dose_subset(wl.phases, wl.plan, n, seed, 0, 2**32 - 1, h_mod=n_batches, h_rem=b)
        t = np.array(t[0], dtype=np.float64)
        totals.append(t.sum())
        tot = t if tot is None else tot + t
        sq = t * t if sq is None else sq + t * t
    mean = tot / n_batches
    var_b = (sq - n_batches * mean * mean) / (n_batches - 1)
    sigma_total = math.sqrt(n_batches * np.var(totals, ddof=1))
    return tot, np.sqrt(np.maximum(var_b, 0.0) * n_batches), sigma_total


def dose_parity(test_tally, orc_tally, orc_sigma, label=None):
    """(pass fraction, relative total-energy difference, mean and RMS of
    dD / sigma_diff over the voxels above 10 % of the maximum, voxel count)."""
    g = np.asarray(test_tally, dtype=np.float64)
    o = np.asarray(orc_tally, dtype=np.float64)
    dmax = o.max()
    sel = o > 0.1 * dmax
    d = g[sel] - o[sel]
    sig = math.sqrt(2.0) * np.asarray(orc_sigma)[sel]
    ok = (np.abs(d) <= 0.01 * dmax) | (np.abs(d) <= 3.0 * sig)
    frac = float(ok.mean())
    z = d / np.maximum(sig, 1e-30)
    e_rel = abs(g.sum() - o.sum()) / o.sum()
    zm, zr = float(z.mean()), float(np.sqrt(np.mean(z * z)))
    if label:
        say(label, f"voxels>0.1Dmax={int(sel.sum())} pass={frac:.5f} dE={e_rel:.2e} "
                   f"mean z={zm:+.3f} rms z={zr:.3f}")
    return frac, e_rel, zm, zr, int(sel.sum())


def calibration(name):
    with open(os.path.join(HERE, "golden", "pass_fractions.json")) as f:
        return json.load(f)[name]


def independent_bar(name):
    """Lowest acceptable pass fraction of an independent-seed comparison of
    the named case: the oracle-vs-oracle mean minus 3 standard errors, the
    larger of the binomial one of a single comparison and the spread of the
    oracle pairs."""
    c = calibration(name)
    f, n = c["mean"], c["voxels"]
    se = max(math.sqrt(f * (1.0 - f) / n), c["sd"])
    return f - 3.0 * se
