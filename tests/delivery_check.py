"""Comparison of a delivery simulation with the oracle's (`oracle.delivery`).

Both draw their Gaussians by Box-Muller in FP64, but with different
logarithm and cosine implementations (the device's and the host's libm), so
a draw may differ in its last bit.  Everything downstream is the same FP64
walk, so a timeline agrees with the oracle's exactly in its MU per (spot,
phase) and its fill count unless one of its decisions sat at a near tie
(the oracle logs the smallest relative gap of every comparison a last-bit
difference could flip); its end time agrees to 1e-12 relative."""
import numpy as np

TIE = 1e-10          # a decision whose operands differ by less than this (relative) may flip
TIME_RTOL = 1e-12


def compare(got, want, spots, n_fields, max_flips=0):
    """Returns the number of (trial, field) timelines that differ; each of
    them must carry a near-tie decision in the oracle's log."""
    n_trials = want["mu"].shape[0]
    flips = []
    for f in range(n_fields):
        idx = np.flatnonzero(spots["field"] == f)
        for t in range(n_trials):
            if (np.array_equal(got["mu"][t, idx], want["mu"][t, idx])
                    and got["fills"][t, f] == want["fills"][t, f]):
                a, b = float(got["time"][t, f]), float(want["time"][t, f])
                assert abs(a - b) <= TIME_RTOL * max(abs(b), 1.0), (t, f, a, b)
            else:
                assert want["margin"][t, f] < TIE, \
                    f"trial {t} field {f} differs with no near-tie decision (margin {want['margin'][t, f]:.3e})"
                flips.append((t, f))
    assert len(flips) <= max_flips, flips
    return len(flips)


def same(got, want):
    """Bit-identical (two runs of one implementation, or draws multiplied by 0)."""
    assert np.array_equal(got["fills"], want["fills"])
    assert np.array_equal(got["time"], want["time"])
    assert np.array_equal(got["mu"], want["mu"])
